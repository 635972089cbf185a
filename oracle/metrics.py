"""Resampling-quality measures of the paper's Section 5.1 (test infrastructure).

offspring count o_k^(i)  : number of particles that chose particle i as ancestor
SE(o_k)                  : sum_i (o_k^(i) - N w_i / sum_j w_j)^2
MSE(o)                   : mean of SE over K offspring vectors; reported as MSE/N
||Bias(o)||^2            : sum_i (mean_k o_k^(i) - N w_i / sum_j w_j)^2
bias contribution        : ||Bias||^2 / MSE   (eq. (bias-contrib))

The paper writes the bias term with a hatted weight; it is read here as the
same weight w (there is only one weight vector per experiment).
"""
from __future__ import annotations

import numpy as np


def offspring(anc: np.ndarray, n: int) -> np.ndarray:
    """o^(i) = #{particles whose ancestor is i}."""
    return np.bincount(np.asarray(anc, dtype=np.int64), minlength=n)[:n]


def expected_offspring(w: np.ndarray) -> np.ndarray:
    w = np.asarray(w, dtype=np.float64)
    return w.size * w / w.sum()


def squared_error(o: np.ndarray, w: np.ndarray) -> float:
    d = np.asarray(o, dtype=np.float64) - expected_offspring(w)
    return float(np.dot(d, d))


class QualityAccumulator:
    """Accumulates K offspring vectors of one weight sequence."""

    def __init__(self, w: np.ndarray):
        self.w = np.asarray(w)
        self.n = self.w.size
        self.expected = expected_offspring(self.w)
        self.k = 0
        self.se_sum = 0.0
        self.o_sum = np.zeros(self.n, dtype=np.float64)
        self.se_list = []
        self.o_sq_sum = np.zeros(self.n, dtype=np.float64)

    def add(self, anc: np.ndarray) -> None:
        o = offspring(anc, self.n).astype(np.float64)
        d = o - self.expected
        se = float(np.dot(d, d))
        self.se_sum += se
        self.se_list.append(se)
        self.o_sum += o
        self.o_sq_sum += o * o
        self.k += 1

    def mean_offspring(self) -> np.ndarray:
        return self.o_sum / self.k

    def variance_sum(self) -> float:
        """sum_i of the sample variance of o^(i) over the K vectors (1/(K-1))."""
        m = self.o_sum / self.k
        return float(np.sum((self.o_sq_sum - self.k * m * m) / (self.k - 1)))

    def bias_sq_debiased(self) -> float:
        """||Bias||^2 less the part that the finite K adds to it: the squared
        distance of the K-sample mean from the expected offspring exceeds the
        squared bias by (sum_i Var o^(i)) / K on average."""
        return self.bias_sq() - self.variance_sum() / self.k

    def mse(self) -> float:
        return self.se_sum / self.k

    def mse_over_n(self) -> float:
        return self.mse() / self.n

    def bias_sq(self) -> float:
        d = self.o_sum / self.k - self.expected
        return float(np.dot(d, d))

    def bias_contribution(self) -> float:
        return self.bias_sq() / self.mse()

    def mse_over_n_stderr(self) -> float:
        se = np.asarray(self.se_list) / self.n
        if se.size < 2:
            return float("inf")
        return float(se.std(ddof=1) / np.sqrt(se.size))
