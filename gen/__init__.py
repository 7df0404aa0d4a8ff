"""Seeded synthetic inputs for the structure-function path.

This package only draws input frames and lag lists. It holds none of the
analysis arithmetic (no forward transform of the frames, no pair
differences, no binning): both the FP64 oracle and the HIP path receive the
same frames from here and nothing else.
"""
from .lags import log_spaced_lags, power_of_two_lags
from .frames import make_stack, cosine_stack
from .configs import CONFIGS, config, batch_workload

__all__ = ["log_spaced_lags", "power_of_two_lags", "make_stack",
           "cosine_stack", "CONFIGS", "config", "batch_workload"]
