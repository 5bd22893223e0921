"""Seeded synthetic inputs shaped like the paper's clustering workloads.

The paper clusters up to 2,000,000 records with up to 25 features
(Abstract; Introduction; Problem statement) but names no dataset, so every
input here is synthetic: Gaussian mixtures (the clustered structure that the
nearest-neighbour method is meant to find) and small-integer grids (heavy
duplicate and equal-distance structure).

This module holds no part of the clustering method: it only draws numbers.
Both the CPU oracle and the GPU library consume its arrays, which is why it
lives on its own.  Every draw goes through ``numpy.random.default_rng`` seeded
from a ``SeedSequence``; draws happen in a fixed order (centres, shapes,
weights, counts, points, noise, permutation), arithmetic is FP64 and the
result is cast to FP32 once, at the end.

Workloads (N points x D features, FP32, row-major [N][D]):

* ``blobs8``: N=4096, D=8, 8 isotropic blobs, centres U[0,10]^8, sigma=0.5,
  exactly N/8 points per blob, then a seeded permutation.
* ``mixture64``: N=262,144, D=25, 64 isotropic Gaussians with centres
  U[0,1]^25, per-cluster sigma log-uniform in [0.005, 0.05], Dirichlet(1)
  weights (multinomial counts), plus round(0.05 N) uniform U[0,1]^25 noise
  points; N is the total.
* ``aniso500``: N=2,000,000, D=25, 500 anisotropic Gaussians (random
  rotation from a sign-fixed QR of a Gaussian matrix, axis sigma
  log-uniform in [0.002, 0.03], centres U[0,1]^25, Dirichlet(1) weights),
  then per-feature min-max scaling to [0, 1] in FP64.
* ``batch256``: 256 instances, N log-uniform in [1024, 65536], D uniform in
  {4..25}, each a mixture of U{4..64} isotropic Gaussians (sigma log-uniform
  in [0.005, 0.05], centres U[0,1]^D, Dirichlet(1) weights); instance i is
  drawn from ``SeedSequence(seed).spawn(256)[i]``.
* ``int16grid``: N=2,000,000, D=25, integers uniform in 0..15 stored as
  FP32 (exact), so squared distances are small integers with massive ties.

Every generator takes ``n`` (and the others their natural knobs) so tests can
draw the same recipe at reduced size.
"""
from __future__ import annotations

import hashlib

import numpy as np

__all__ = [
    "blobs8",
    "mixture64",
    "aniso500",
    "batch256",
    "int16grid",
    "sha256",
    "WORKLOADS",
]


def _rng(seed):
    if isinstance(seed, np.random.SeedSequence):
        return np.random.default_rng(seed)
    return np.random.default_rng(np.random.SeedSequence(int(seed)))


def _log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=size))


def _counts(rng, n, weights):
    return rng.multinomial(n, weights)


def sha256(x: np.ndarray) -> str:
    """SHA-256 of the array's bytes (C order)."""
    return hashlib.sha256(np.ascontiguousarray(x).tobytes()).hexdigest()


def blobs8(seed: int = 0, n: int = 4096, d: int = 8, k: int = 8,
           sigma: float = 0.5, box: float = 10.0):
    """Isotropic blobs; returns (X float32 [n][d], generating labels int64 [n])."""
    rng = _rng(seed)
    centres = rng.uniform(0.0, box, size=(k, d))
    per = np.full(k, n // k, dtype=np.int64)
    per[: n - per.sum()] += 1
    pts, lab = [], []
    for c in range(k):
        pts.append(centres[c] + sigma * rng.standard_normal((per[c], d)))
        lab.append(np.full(per[c], c, dtype=np.int64))
    X = np.concatenate(pts)
    y = np.concatenate(lab)
    p = rng.permutation(n)
    return X[p].astype(np.float32), y[p]


def mixture64(seed: int = 0, n: int = 262_144, d: int = 25, k: int = 64,
              noise_frac: float = 0.05):
    """Isotropic Gaussian mixture plus uniform noise; returns (X, labels),
    label -1 marks a noise point."""
    rng = _rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(k, d))
    sig = _log_uniform(rng, 0.005, 0.05, k)
    w = rng.dirichlet(np.ones(k))
    n_noise = int(round(noise_frac * n))
    cnt = _counts(rng, n - n_noise, w)
    pts, lab = [], []
    for c in range(k):
        pts.append(centres[c] + sig[c] * rng.standard_normal((cnt[c], d)))
        lab.append(np.full(cnt[c], c, dtype=np.int64))
    pts.append(rng.uniform(0.0, 1.0, size=(n_noise, d)))
    lab.append(np.full(n_noise, -1, dtype=np.int64))
    X = np.concatenate(pts)
    y = np.concatenate(lab)
    p = rng.permutation(n)
    return X[p].astype(np.float32), y[p]


def _rotation(rng, d):
    g = rng.standard_normal((d, d))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def aniso500(seed: int = 0, n: int = 2_000_000, d: int = 25, k: int = 500):
    """Anisotropic Gaussian mixture min-max scaled to [0,1]; returns (X, labels)."""
    rng = _rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(k, d))
    rots = [_rotation(rng, d) for _ in range(k)]
    axis = _log_uniform(rng, 0.002, 0.03, (k, d))
    w = rng.dirichlet(np.ones(k))
    cnt = _counts(rng, n, w)
    X = np.empty((n, d), dtype=np.float64)
    y = np.empty(n, dtype=np.int64)
    off = 0
    for c in range(k):
        z = rng.standard_normal((cnt[c], d)) * axis[c][None, :]
        X[off: off + cnt[c]] = centres[c] + z @ rots[c].T
        y[off: off + cnt[c]] = c
        off += cnt[c]
    lo = X.min(axis=0)
    hi = X.max(axis=0)
    X = (X - lo) / np.where(hi > lo, hi - lo, 1.0)
    p = rng.permutation(n)
    return X[p].astype(np.float32), y[p]


def int16grid(seed: int = 0, n: int = 2_000_000, d: int = 25, levels: int = 16):
    """Integer features uniform in 0..levels-1, stored exactly as FP32."""
    rng = _rng(seed)
    return rng.integers(0, levels, size=(n, d)).astype(np.float32)


def batch256(seed: int = 0, count: int = 256, n_lo: int = 1024,
             n_hi: int = 65536, d_lo: int = 4, d_hi: int = 25,
             with_components: bool = False):
    """List of ``count`` independent mixture instances of uneven N and D.

    With ``with_components`` the result is ``(instances, ks)``, ks[i] being
    the number of mixture components instance i was drawn from (the draws
    are the same either way)."""
    out = []
    ks = []
    for ss in np.random.SeedSequence(int(seed)).spawn(count):
        rng = np.random.default_rng(ss)
        n = int(round(float(_log_uniform(rng, n_lo, n_hi, 1)[0])))
        d = int(rng.integers(d_lo, d_hi + 1))
        k = int(rng.integers(4, 65))
        centres = rng.uniform(0.0, 1.0, size=(k, d))
        sig = _log_uniform(rng, 0.005, 0.05, k)
        w = rng.dirichlet(np.ones(k))
        cnt = _counts(rng, n, w)
        pts = [centres[c] + sig[c] * rng.standard_normal((cnt[c], d))
               for c in range(k)]
        X = np.concatenate(pts)
        X = X[rng.permutation(n)]
        out.append(X.astype(np.float32))
        ks.append(k)
    if with_components:
        return out, ks
    return out


WORKLOADS = {
    "blobs8": blobs8,
    "mixture64": mixture64,
    "aniso500": aniso500,
    "int16grid": int16grid,
}
