"""Seeded initial parameters of the 32 -> 64 -> 64 -> 12 schedule network.

He-uniform weights (He et al., ICCV 2015: variance 2 / fan_in, drawn as
U(-sqrt(6 / fan_in), +sqrt(6 / fan_in))), zero biases, in the flat layout
W1[64,32], b1[64], W2[64,64], b2[64], W3[12,64], b3[12] (7,052 values).
Returned as float32, the precision the GPU trains in; the oracle widens it.
"""
import numpy as np

from .memcpy import rng

LAYERS = [(64, 32), (64, 64), (12, 64)]


def he_uniform(seed_batch: int = 0) -> np.ndarray:
    g = rng(30, seed_batch)
    parts = []
    for fan_out, fan_in in LAYERS:
        lim = np.sqrt(6.0 / fan_in)
        parts.append(g.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)
