"""Macroscopic strain histories for strain-controlled cyclic loading."""
import numpy as np


def triangular_waveform(amplitude, ratio, cycles, incs_per_cycle, rate=1e-3):
    """Increments of the loading-axis macro strain for a triangular cycle starting at 0.

    ratio = -1: 0 -> +a -> 0 -> -a -> 0 per cycle (a/(n/4) per increment);
    ratio =  0: 0 -> +a -> 0 per cycle (a/(n/2) per increment).
    Returns (deps, dt): arrays of length cycles*incs_per_cycle, with
    dt = |deps| / rate (strain rate ``rate`` in 1/s).
    """
    n = int(incs_per_cycle)
    if ratio == -1:
        if n % 4:
            raise ValueError("fully reversed cycles need a multiple of 4 increments")
        q = n // 4
        step = amplitude / q
        one = [step] * q + [-step] * (2 * q) + [step] * q
    elif ratio == 0:
        if n % 2:
            raise ValueError("R=0 cycles need an even number of increments")
        q = n // 2
        step = amplitude / q
        one = [step] * q + [-step] * q
    else:
        raise ValueError("strain ratio must be -1 or 0")
    deps = np.array(one * int(cycles), dtype=np.float64)
    dt = np.abs(deps) / rate
    return deps, dt
