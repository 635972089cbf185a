"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no resampling arithmetic: only the weight and state
generators of the paper's experiments (Section 5, eq. (distribution)) and the
workload recipes built from them. Both the HIP path and the CPU oracle are fed
the exact same fp32 bytes from here.

Gaussian-likelihood weights: x_i ~ N(0,1) in fp64 from numpy's PCG64 seeded
with 12345 + q, then w_i = exp(-(x_i - y)^2 / 2) rounded once to fp32. The
paper's constant factor 1/sqrt(2 pi) is dropped: the resamplers and the
iteration count B are invariant to a common scale of the weights.
"""
from __future__ import annotations

import numpy as np

WEIGHT_SEED_BASE = 12345
STATE_SEED_BASE = 54321
BATCH_SEED = 777
SERVE_SEED = 999


def gaussian_x(n: int, q: int = 0) -> np.ndarray:
    return np.random.Generator(np.random.PCG64(WEIGHT_SEED_BASE + q)).standard_normal(n)


def gaussian_weights(n: int, y: float, q: int = 0) -> np.ndarray:
    """fp32 weights w_i = exp(-(x_i - y)^2 / 2), x_i ~ N(0,1) (eq. (distribution))."""
    x = gaussian_x(n, q)
    return np.exp(-0.5 * (x - y) ** 2).astype(np.float32)


def gaussian_weights_and_states(n: int, y: float, d: int, q: int = 0):
    """Weights plus fp32 AoS states [n, d]; state[:, 0] = x, other dims N(0,1)."""
    x = gaussian_x(n, q)
    w = np.exp(-0.5 * (x - y) ** 2).astype(np.float32)
    st = np.empty((n, d), dtype=np.float32)
    st[:, 0] = x.astype(np.float32)
    if d > 1:
        g = np.random.Generator(np.random.PCG64(STATE_SEED_BASE + q))
        st[:, 1:] = g.standard_normal((n, d - 1)).astype(np.float32)
    return w, st


def gamma_weights(n: int, alpha: float, q: int = 0) -> np.ndarray:
    """Gamma(alpha, rate 1) weights (eq. (gammaEq)); fp32."""
    g = np.random.Generator(np.random.PCG64(WEIGHT_SEED_BASE + 1000 + q))
    return g.gamma(alpha, 1.0, n).astype(np.float32)


def uniform_weights(n: int, value: float = 0.5) -> np.ndarray:
    return np.full(n, value, dtype=np.float32)


def single_spike_weights(n: int, p: int, value: float = 1.0) -> np.ndarray:
    w = np.zeros(n, dtype=np.float32)
    w[p] = value
    return w


def two_level_weights(n: int, p: int, c: float) -> np.ndarray:
    """w_p = 1, every other weight c."""
    w = np.full(n, c, dtype=np.float32)
    w[p] = 1.0
    return w


def random_states(n: int, d: int, seed: int) -> np.ndarray:
    return np.random.Generator(np.random.PCG64(seed)).standard_normal((n, d)).astype(np.float32)


# ---------------------------------------------------------------------------
# Workload recipes
# ---------------------------------------------------------------------------

def batch_filters(count: int = 512, n_lo_log2: float = 10.0, n_hi_log2: float = 18.0, seed: int = BATCH_SEED):
    """Filter sizes N_f = round(2^U(lo, hi)) and y_f ~ U[0, 4] for the batched workload."""
    g = np.random.Generator(np.random.PCG64(seed))
    n = np.rint(2.0 ** g.uniform(n_lo_log2, n_hi_log2, count)).astype(np.int64)
    y = g.uniform(0.0, 4.0, count)
    return n, y


def serving_requests(count: int, rate_per_s: float, n_lo_log2: float = 12.0, n_hi_log2: float = 22.0,
                     seed: int = SERVE_SEED):
    """Poisson arrivals (exponential gaps at the given rate), sizes and y per request."""
    g = np.random.Generator(np.random.PCG64(seed))
    gaps = g.exponential(1.0 / rate_per_s, count)
    t = np.cumsum(gaps)
    n = np.rint(2.0 ** g.uniform(n_lo_log2, n_hi_log2, count)).astype(np.int64)
    y = g.uniform(0.0, 4.0, count)
    return t, n, y



# ---------------------------------------------------------------------------
# The SIR application's synthetic data (Section 7)
# ---------------------------------------------------------------------------
SIR_SEED = 2021


def sir_truth(T: int = 100, trajectories: int = 16, seed: int = SIR_SEED):
    """Ground-truth states x_0..x_T and measurements z_0..z_T of the model of
    Section 7 (fp64): x_t = x_{t-1}/2 + 25 x_{t-1}/(1 + x_{t-1}^2) +
    8 cos(1.2 t) + v, v ~ N(0, 10); z_t = x_t^2/20 + n, n ~ N(0, 1); x_0 ~ N(0, 5)."""
    g = np.random.Generator(np.random.PCG64(seed))
    x = np.empty((trajectories, T + 1))
    z = np.empty((trajectories, T + 1))
    x[:, 0] = g.normal(0.0, np.sqrt(5.0), trajectories)
    z[:, 0] = x[:, 0] ** 2 / 20.0 + g.normal(0.0, 1.0, trajectories)
    for t in range(1, T + 1):
        xp = x[:, t - 1]
        x[:, t] = xp / 2.0 + 25.0 * xp / (1.0 + xp * xp) + 8.0 * np.cos(1.2 * t) + g.normal(0.0, np.sqrt(10.0),
                                                                                             trajectories)
        z[:, t] = x[:, t] ** 2 / 20.0 + g.normal(0.0, 1.0, trajectories)
    return x, z


def sir_initial_particles(n: int, run: int, seed: int = SIR_SEED + 1) -> np.ndarray:
    """Initial particles of run `run`, drawn from the prior N(0, 5) (fp32)."""
    g = np.random.Generator(np.random.PCG64(seed + 7919 * run))
    return g.normal(0.0, np.sqrt(5.0), n).astype(np.float32)


def sir_initial_particles_torch(runs: int, n: int, device, seed: int = SIR_SEED + 2):
    """Initial particles of `runs` runs drawn from the prior N(0, 5) by torch's
    seeded generator on `device` (fp32, [runs, n]): for experiments too large
    to draw on the host."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    x = torch.randn((runs, n), generator=g, device=device, dtype=torch.float32)
    return x.mul_(float(np.sqrt(5.0)))
