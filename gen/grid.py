"""Spatially correlated AR(1) series on a lat/lon grid, with anomaly patches.

Recipe (the inputs are synthetic stand-ins for gridded precipitation fields):

* Grid of G x G cells; node id = row * G + col; distances between cells are
  Euclidean in cell units (no wrap-around).
* Each time step draws one Gaussian random field with unit variance and
  covariance exp(-dist / ell) (ell = 3 cells).  Fields come from circulant
  embedding on a (2G) x (2G) torus: the torus covariance's spectrum is taken
  by FFT, negative eigenvalues are clipped to zero, and the complex-FFT trick
  yields two independent fields per transform.  The top-left G x G block is
  kept.
* Each node carries an AR(1) series x_t = phi * x_{t-1} + e_t (phi = 0.7),
  started from its stationary law (x_0 = e_0 / sqrt(1 - phi^2)), where e_t is
  the field of time step t.  So the innovations are spatially correlated.
* An anomaly patch is a square block of cells whose series is negated
  ("correlation flipped") from an onset time onward.

All randomness comes from numpy's PCG64 generator seeded with the given seeds,
so an input is a pure function of its parameters.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

PHI = 0.7
ELL = 3.0

# Named workloads.  k = number of random projections, d = chain depth
# (number of stored levels; 0 = adaptive), prec = chain arithmetic.
CONFIGS = {
    "C1": dict(G=16, T=120, patches=1, patch_size=3, k=32, depth=8, prec="fp64"),
    "C2": dict(G=64, T=240, patches=4, patch_size=4, k=128, depth=0, prec="fp32"),
    "C3": dict(G=128, T=240, patches=4, patch_size=4, k=256, depth=0, prec="bf16"),
    "C4": dict(G=96, T=120, n_snap=24, stride=30, n_min=1024, n_max=8192,
               patch_size=4, onsets=(8, 16), k=128, depth=0, prec="bf16"),
    "C5": dict(G=256, T=360, patches=4, patch_size=8, k=200, depth=0, prec="bf16"),
}

DATA_SEED = 1
PATCH_SEED = 11
PROJ_SEED = 7


def _sqrt_spectrum(G: int, ell: float) -> np.ndarray:
    """Square root of the (clipped) circulant spectrum, scaled for fft2."""
    M = 2 * G
    d = np.arange(M)
    d = np.minimum(d, M - d).astype(np.float64)
    r = np.sqrt(d[:, None] ** 2 + d[None, :] ** 2)
    base = np.exp(-r / ell)
    lam = np.fft.fft2(base).real
    lam = np.clip(lam, 0.0, None)
    return np.sqrt(lam / float(M * M))


def _fields(rng: np.random.Generator, G: int, count: int, ell: float) -> np.ndarray:
    """`count` independent unit-variance fields, shape (count, G*G)."""
    sq = _sqrt_spectrum(G, ell)
    M = 2 * G
    out = np.empty((count, G * G), dtype=np.float64)
    t = 0
    while t < count:
        xi = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
        f = np.fft.fft2(sq * xi)
        out[t] = f.real[:G, :G].reshape(-1)
        t += 1
        if t < count:
            out[t] = f.imag[:G, :G].reshape(-1)
            t += 1
    return out


def ar1_grid_series(G: int, length: int, seed: int, phi: float = PHI,
                    ell: float = ELL) -> np.ndarray:
    """AR(1) series for every cell of a G x G grid: array (G*G, length)."""
    rng = np.random.default_rng(seed)
    e = _fields(rng, G, length, ell)            # (length, n)
    x = np.empty((G * G, length), dtype=np.float64)
    prev = e[0] / np.sqrt(1.0 - phi * phi)
    x[:, 0] = prev
    for t in range(1, length):
        prev = phi * prev + e[t]
        x[:, t] = prev
    return x


def place_patches(G: int, count: int, size: int, seed: int) -> List[Tuple[int, int]]:
    """Top-left corners of `count` non-overlapping size x size patches."""
    rng = np.random.default_rng(seed)
    taken = np.zeros((G, G), dtype=bool)
    corners: List[Tuple[int, int]] = []
    tries = 0
    while len(corners) < count:
        tries += 1
        if tries > 100000:
            raise ValueError("cannot place patches")
        r, c = (int(v) for v in rng.integers(0, G - size + 1, size=2))
        if taken[r:r + size, c:c + size].any():
            continue
        taken[r:r + size, c:c + size] = True
        corners.append((r, c))
    return corners


def patch_nodes(G: int, corners: Sequence[Tuple[int, int]], size: int) -> np.ndarray:
    ids = [(r + i) * G + (c + j) for (r, c) in corners
           for i in range(size) for j in range(size)]
    return np.array(sorted(ids), dtype=np.int64)


@dataclass
class GridPair:
    """Two snapshots' node series (n x T each, row-major float64)."""
    G: int
    T: int
    X0: np.ndarray
    X1: np.ndarray
    gid: np.ndarray               # global node ids (identity here)
    anomalous: np.ndarray         # node ids whose series flip in window 1

    @property
    def n(self) -> int:
        return self.G * self.G


def make_pair(G: int, T: int, patches: int, patch_size: int,
              data_seed: int = DATA_SEED, patch_seed: int = PATCH_SEED) -> GridPair:
    """Windows [0,T) and [T,2T) of one series; patches negated in the second."""
    x = ar1_grid_series(G, 2 * T, data_seed)
    corners = place_patches(G, patches, patch_size, patch_seed)
    anom = patch_nodes(G, corners, patch_size)
    X0 = np.ascontiguousarray(x[:, :T])
    X1 = np.ascontiguousarray(x[:, T:])
    X1[anom] *= -1.0
    return GridPair(G=G, T=T, X0=X0, X1=X1,
                    gid=np.arange(G * G, dtype=np.int32), anomalous=anom)


def make_config_pair(name: str, **over) -> GridPair:
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    return make_pair(cfg["G"], cfg["T"], cfg["patches"], cfg["patch_size"])


@dataclass
class GridSequence:
    """Snapshots on random node subsets of one grid (uneven sizes)."""
    G: int
    T: int
    X: List[np.ndarray] = field(default_factory=list)     # n_t x T each
    gid: List[np.ndarray] = field(default_factory=list)   # sorted int32 ids
    anomalous: List[np.ndarray] = field(default_factory=list)


def make_sequence(G: int = 96, T: int = 120, n_snap: int = 24, stride: int = 30,
                  n_min: int = 1024, n_max: int = 8192, patch_size: int = 4,
                  onsets: Sequence[int] = (8, 16), data_seed: int = DATA_SEED,
                  patch_seed: int = PATCH_SEED) -> GridSequence:
    """Sliding windows [stride*t, stride*t + T) over uneven random subsets.

    Patch p (one per onset) has its series negated from time stride*onset_p
    onward; snapshot t keeps a uniformly random subset of n_t cells,
    n_t ~ U{n_min..n_max}.
    """
    length = T + (n_snap - 1) * stride
    x = ar1_grid_series(G, length, data_seed)
    corners = place_patches(G, len(onsets), patch_size, patch_seed)
    flipped = []
    for (corner, onset) in zip(corners, onsets):
        ids = patch_nodes(G, [corner], patch_size)
        x[ids, stride * onset:] *= -1.0
        flipped.append((ids, onset))
    rng = np.random.default_rng(patch_seed + 1000)
    seq = GridSequence(G=G, T=T)
    for t in range(n_snap):
        n_t = int(rng.integers(n_min, n_max + 1))
        ids = np.sort(rng.choice(G * G, size=n_t, replace=False)).astype(np.int32)
        seq.gid.append(ids)
        seq.X.append(np.ascontiguousarray(x[ids, stride * t: stride * t + T]))
        an = [i for (pid, onset) in flipped if t >= onset - 3 for i in pid]
        seq.anomalous.append(np.array(sorted(set(an)), dtype=np.int64))
    return seq
