"""Seeded initial weights of the CNN refiner (inputs to both the GPU path and
the oracle): He-uniform weights, zero biases.  Holds no network arithmetic."""

from __future__ import annotations

import numpy as np

# (fan_in, count) of each parameter tensor, in the order the network stores them:
# conv1..conv4 (weights [co][3][3][ci], biases [co]), fc1 ([10][2048], [10]), fc2 ([2][10], [2])
LAYOUT = (
    (9, 32 * 9), (0, 32),
    (288, 32 * 288), (0, 32),
    (288, 32 * 288), (0, 32),
    (288, 32 * 288), (0, 32),
    (2048, 10 * 2048), (0, 10),
    (10, 2 * 10), (0, 2),
)
N_PARAMS = sum(c for _, c in LAYOUT)


def init_params(seed: int = 0) -> np.ndarray:
    """Flat float32 vector of N_PARAMS parameters."""
    rng = np.random.default_rng(np.random.SeedSequence([220903883, 5, seed]))
    out = []
    for fan_in, count in LAYOUT:
        if fan_in == 0:
            out.append(np.zeros(count))
        else:
            lim = np.sqrt(6.0 / fan_in)
            out.append(rng.uniform(-lim, lim, count))
    return np.concatenate(out).astype(np.float32)
