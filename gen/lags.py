"""Lag lists used as inputs.

The paper analyses all N-1 delays and suggests, as a cheaper alternative,
delays spread evenly on a logarithmic scale (discussion section, ref. [21]).
The lag list is an input of the analysis; this module only builds such lists.
"""
import math


def log_spaced_lags(tau_max, count):
    """`count` distinct integer lags from 1 to `tau_max`, evenly spaced in log.

    Lag j is round(tau_max ** (j / (count - 1))) with halves rounded up; when
    that is not larger than lag j-1 it is bumped to lag j-1 plus one, so the
    list always has `count` distinct, strictly increasing entries.
    """
    tau_max = int(tau_max)
    count = int(count)
    if count < 1 or tau_max < 1:
        raise ValueError("need tau_max >= 1 and count >= 1")
    if count == 1:
        return [tau_max]
    if count > tau_max:
        raise ValueError("cannot draw more distinct lags than tau_max")
    out = []
    for j in range(count):
        t = int(math.floor(tau_max ** (j / (count - 1)) + 0.5))
        if out and t <= out[-1]:
            t = out[-1] + 1
        out.append(t)
    if out[-1] != tau_max:
        raise ValueError("log-spaced lag rule overshot tau_max")
    return out


def power_of_two_lags(tau_max):
    """1, 2, 4, ... up to and including the largest power of two <= tau_max."""
    out = []
    t = 1
    while t <= tau_max:
        out.append(t)
        t *= 2
    return out
