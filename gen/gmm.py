"""The paper's synthetic data set (Section "Data description", Synthetic
Data): a two-snapshot graph sequence on points of a 2-D mixture of four
Gaussians, with planted anomalous edges between clusters.

A_1(i, j) = exp(-d(i, j)) over the Euclidean distances of the points; A_2 is
the same kernel over the points moved by a little noise, plus (R + R^T) / 2
where R(i, j) is uniform on [0, 1) with probability 0.05 and 0 otherwise.
The anomalous edges are those with R(i, j) != 0 or R(j, i) != 0 whose ends
lie in different clusters.  This kernel defines the data set's input graphs
(the paper gives them this way); the method's own graph construction (the
Gaussian kernel of time series with a median bandwidth) is not here.

The paper does not give the mixture's parameters or the noise level; the
defaults below (unit-variance components at the corners of a square of side
4, noise 0.05) are this data set's reading.
"""

from dataclasses import dataclass

import numpy as np

GMM_SEED = 3


@dataclass
class GmmPair:
    A1: np.ndarray          # n x n weights, zero diagonal
    A2: np.ndarray          # n x n weights, zero diagonal
    labels: np.ndarray      # mixture component of each node
    anomalous: np.ndarray   # n x n bool, symmetric: planted inter-cluster edges


def _kernel(Y: np.ndarray) -> np.ndarray:
    d = np.sqrt(((Y[:, None, :] - Y[None, :, :]) ** 2).sum(-1))
    W = np.exp(-d)
    np.fill_diagonal(W, 0.0)
    return W


def make_gmm_pair(n: int, seed: int = GMM_SEED, side: float = 4.0, noise: float = 0.05,
                  p: float = 0.05) -> GmmPair:
    rng = np.random.default_rng(seed)
    centers = np.array([[0.0, 0.0], [side, 0.0], [0.0, side], [side, side]])
    labels = rng.integers(0, 4, n)
    X1 = centers[labels] + rng.standard_normal((n, 2))
    X2 = X1 + noise * rng.standard_normal((n, 2))
    R = np.where(rng.random((n, n)) < p, rng.random((n, n)), 0.0)
    np.fill_diagonal(R, 0.0)
    A2 = _kernel(X2) + (R + R.T) / 2
    anomalous = ((R != 0) | (R.T != 0)) & (labels[:, None] != labels[None, :])
    return GmmPair(A1=_kernel(X1), A2=A2, labels=labels, anomalous=anomalous)
