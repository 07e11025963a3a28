"""Seeded initial parameters of the learned-guess network (random numbers
only; no arithmetic of the method). Packing as in the library and the
checker: W1 (64 x 6), b1, W2 (64 x 64), b2, W3 (64 x 64), b3, W4 (1 x 64), b4.
Weights are normal with standard deviation sqrt(2 / fan_in), biases zero."""
import numpy as np

SIZES = [(64, 6), (64,), (64, 64), (64,), (64, 64), (64,), (1, 64), (1,)]


def init_params(seed=0, out_scale=0.1):
    rng = np.random.default_rng(seed)
    parts = []
    for k, s in enumerate(SIZES):
        if len(s) == 2:
            std = np.sqrt(2.0 / s[1]) * (out_scale if k == 6 else 1.0)
            parts.append(rng.normal(0.0, std, size=s))
        else:
            parts.append(np.zeros(s))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def random_features(seed, rows):
    """Synthetic feature rows with the ranges of the real ones."""
    rng = np.random.default_rng(seed)
    X = np.empty((rows, 6), dtype=np.float32)
    X[:, 0] = rng.uniform(-8.0, 1.0, rows)
    X[:, 1] = rng.uniform(-1.0, 1.0, rows)
    X[:, 2] = rng.normal(0.0, 0.05, rows)
    d = np.sort(rng.uniform(0.0, 2.5, (rows, 3)), axis=1)
    X[:, 3:] = d
    t = rng.normal(0.0, 0.1, rows).astype(np.float32)
    return X, t
