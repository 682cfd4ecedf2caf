"""Seeded synthetic inputs of the mask producer (the classifier of Sec. 3.2): parameter
vectors, global feature vectors and spectra.  Inputs only: no network arithmetic.

The paper's trained weights are not available; parameters are drawn like a freshly
initialised network (uniform on +-scale/sqrt(fan_in) per layer, weights and biases), then
rounded to float32.  ``scale`` > 1 spreads the output probabilities over (0, 1) so that the
coarse percentile and the threshold cut through varied values.
"""
from __future__ import annotations

import numpy as np

# (out, in) of every layer in parameter order; each layer is W (out x in, row-major) then b.
LAYER_SHAPES = ((64, 26), (64, 64), (128, 33), (64, 128), (128, 128), (128, 128), (64, 128), (1, 64))
NPARAM = sum(o * i + o for o, i in LAYER_SHAPES)

__all__ = ["LAYER_SHAPES", "NPARAM", "mlp_params", "global_features", "spectrum"]


def mlp_params(seed: int, scale: float = 1.0) -> np.ndarray:
    """float32[NPARAM]: every layer's W then b, uniform on +-scale/sqrt(fan_in)."""
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in LAYER_SHAPES:
        lim = scale / np.sqrt(i)
        parts.append(rng.uniform(-lim, lim, size=o * i))
        parts.append(rng.uniform(-lim, lim, size=o))
    return np.concatenate(parts).astype(np.float32)


def global_features(seed: int) -> np.ndarray:
    """float64[30]: a stand-in for f1 .. f30 (standard normal draws)."""
    return np.random.default_rng(seed).standard_normal(30)


def spectrum(seed: int, n: int, radius: float = 2.0) -> np.ndarray:
    """complex128[n]: n points uniform in the disk of the given radius (a stand-in spectrum)."""
    rng = np.random.default_rng(seed)
    r = radius * np.sqrt(rng.uniform(size=n))
    return r * np.exp(2j * np.pi * rng.uniform(size=n))
