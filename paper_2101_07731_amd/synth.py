"""Seeded synthetic workloads for multivariate DTW nearest-neighbour search.

This module only draws inputs; it holds none of the method's arithmetic.
The GPU path and the FP64 oracle are both fed from here.  The paper
measures on 13 UEA/UCR multivariate archives (Sec. 7.1, Table 2); these
generators stand in for them with the shapes named per workload below:

  * random walk: x_0 ~ N(0,1), x_t = x_{t-1} + N(0,1), one per dimension;
  * correlated walk (rho = 0.5): x_p = sqrt(.5) s + sqrt(.5) e_p with s and
    e_p independent walks;
  * z-normalisation per series and dimension in float64 (population std;
    a dimension with std < 1e-12 becomes zeros), then cast to float32
    (the paper normalises its data, Sec. 7.1);
  * "prototype" sets: 8 correlated-walk prototypes; each series is one
    prototype resampled through a monotone piecewise-linear time map
    (8 segments, slopes U[0.9, 1.1], rescaled to the series span, i.e. a
    local stretch of at most 10%), plus N(0, 0.1^2) noise, z-normalised,
    so that every query has close neighbours;
  * smooth curves: per dimension a sum of 4 harmonics with amplitudes
    N(0,1)/k and uniform phases (trajectory prototypes).

All generators use numpy's PCG64 (np.random.default_rng) and return
float32 arrays laid out [series][t][d].
"""
from __future__ import annotations

import numpy as np


def znorm(x: np.ndarray) -> np.ndarray:
    """Per-series, per-dimension z-normalisation of [..., T, D] data (float64 in, float64 out)."""
    x = np.asarray(x, dtype=np.float64)
    mu = x.mean(axis=-2, keepdims=True)
    sd = x.std(axis=-2, keepdims=True)
    out = np.where(sd < 1e-12, 0.0, (x - mu) / np.where(sd < 1e-12, 1.0, sd))
    return out


def random_walks(rng, N, T, D):
    """[N, T, D] independent Gaussian random walks (float64)."""
    return np.cumsum(rng.standard_normal((N, T, D)), axis=1)


def correlated_walks(rng, N, T, D, rho=0.5):
    """[N, T, D] walks sharing a latent walk: sqrt(rho) s + sqrt(1-rho) e_p."""
    s = np.cumsum(rng.standard_normal((N, T, 1)), axis=1)
    e = np.cumsum(rng.standard_normal((N, T, D)), axis=1)
    return np.sqrt(rho) * s + np.sqrt(1.0 - rho) * e


def _time_map(rng, T, segments=8, lo=0.9, hi=1.1):
    """Monotone piecewise-linear map of [0, T-1] onto itself with segment slopes in [lo, hi]."""
    slopes = rng.uniform(lo, hi, size=segments)
    t = np.arange(T, dtype=np.float64)
    seg = np.minimum((t * segments / max(T, 1)).astype(np.int64), segments - 1)
    step = slopes[seg]
    tau = np.concatenate([[0.0], np.cumsum(step[:-1])])
    if tau[-1] > 0:
        tau = tau * (T - 1) / tau[-1]
    return tau


def prototype_set(rng, N, T, D, n_proto=8, noise=0.1, protos=None, rho=0.5):
    """N warped noisy copies of n_proto correlated-walk prototypes -> (series [N,T,D] f64, labels [N])."""
    if protos is None:
        protos = znorm(correlated_walks(rng, n_proto, T, D, rho))
    labels = rng.integers(0, protos.shape[0], size=N)
    out = np.empty((N, T, D), dtype=np.float64)
    grid = np.arange(T, dtype=np.float64)
    for k in range(N):
        tau = _time_map(rng, T)
        p = protos[labels[k]]
        for d in range(D):
            out[k, :, d] = np.interp(tau, grid, p[:, d])
        out[k] += noise * rng.standard_normal((T, D))
    return znorm(out), labels


def smooth_curves(rng, N, T, D, harmonics=4):
    """[N, T, D] smooth closed curves: per dimension a sum of harmonics k = 1..h with amplitude
    N(0,1)/k and a uniform phase, z-normalised (pen-trajectory-like paths)."""
    t = np.arange(T, dtype=np.float64) / T
    k = np.arange(1, harmonics + 1, dtype=np.float64)
    amp = rng.standard_normal((N, D, harmonics)) / k
    ph = rng.uniform(0.0, 2.0 * np.pi, size=(N, D, harmonics))
    out = np.einsum("ndh,ndht->ntd", amp, np.sin(2.0 * np.pi * k[None, None, :, None] * t + ph[..., None]))
    return znorm(out)


def _f32(x):
    return np.ascontiguousarray(x, dtype=np.float32)


# --------------------------------------------------------------- workloads --

def plain_knn(nq=64, nc=256, T=64, D=3, seed=1):
    """Plain 1-NN workload: independent random walks per dimension, z-normalised.
    Full size: 64 queries x 256 references, length 64, d = 3, window 10%."""
    rq = np.random.default_rng(2000 + seed)
    rc = np.random.default_rng(1000 + seed)
    Q = _f32(znorm(random_walks(rq, nq, T, D)))
    Cs = _f32(znorm(random_walks(rc, nc, T, D)))
    return Q, Cs


def cascade_knn(nq=1000, nc=10000, T=256, D=8, seed=2, n_proto=8):
    """Pruned 1-NN workload: prototype sets of correlated (rho=.5) walks.
    Full size: 1000 queries x 10000 references, length 256, d = 8,
    windows 5/10/20%.  Queries and references share the prototypes."""
    rp = np.random.default_rng(3000 + seed)
    protos = znorm(correlated_walks(rp, n_proto, T, D))
    rq = np.random.default_rng(2000 + seed)
    rc = np.random.default_rng(1000 + seed)
    Q, _ = prototype_set(rq, nq, T, D, protos=protos)
    Cs, _ = prototype_set(rc, nc, T, D, protos=protos)
    return _f32(Q), _f32(Cs)


def trajectory_knn(nq=1000, nc=10000, T=182, D=3, seed=6, n_proto=20, noise=0.5):
    """Trajectory 1-NN workload, the shape of a pen-trajectory archive (d = 3,
    length 182): 20 prototype classes of smooth curves (smooth_curves, 4
    harmonics), each series a prototype through a random monotone time map plus
    N(0, 0.5^2) noise, z-normalised.  The points of such series lie near curves
    that run across the dimensions, so the per-dimension envelopes of LB_MV are
    loose where the point-clustering boxes of LB_PC are not.
    Full size: 1000 queries x 10000 references, window 10%."""
    rp = np.random.default_rng(3000 + seed)
    protos = smooth_curves(rp, n_proto, T, D)
    rq = np.random.default_rng(2000 + seed)
    rc = np.random.default_rng(1000 + seed)
    Q, _ = prototype_set(rq, nq, T, D, protos=protos, noise=noise)
    Cs, _ = prototype_set(rc, nc, T, D, protos=protos, noise=noise)
    return _f32(Q), _f32(Cs)


def long_knn(nq=200, nc=2000, T=1024, D=16, seed=3):
    """Long multivariate series: correlated walks, z-normalised.
    Full size: 200 queries x 2000 references, length 1024, d = 16, window 10%."""
    rq = np.random.default_rng(2000 + seed)
    rc = np.random.default_rng(1000 + seed)
    Q = _f32(znorm(correlated_walks(rq, nq, T, D)))
    Cs = _f32(znorm(correlated_walks(rc, nc, T, D)))
    return Q, Cs


DIMS_RAGGED = (2, 4, 8, 16, 32)


def ragged_pairs(npairs=4096, tmin=64, tmax=2048, dims=DIMS_RAGGED, seed=4):
    """Uneven pairs: lengths uniform in [tmin, tmax] (independent for x and y),
    d drawn from `dims` per pair (shared by both series); correlated walks,
    z-normalised.  -> (xs, ys): lists of float32 [T, d] arrays."""
    rng = np.random.default_rng(3000 + seed)
    xs, ys = [], []
    for _ in range(npairs):
        D = int(rng.choice(dims))
        m = int(rng.integers(tmin, tmax + 1))
        n = int(rng.integers(tmin, tmax + 1))
        xs.append(_f32(znorm(correlated_walks(rng, 1, m, D))[0]))
        ys.append(_f32(znorm(correlated_walks(rng, 1, n, D))[0]))
    return xs, ys


def ragged_banks(nq=256, nc_per_bank=4096, tmin=64, tmax=2048, dims=DIMS_RAGGED, seed=4):
    """Uneven 1-NN: one reference bank per d in `dims` (lengths uniform in
    [tmin, tmax]); each query draws d and a length and searches the bank of
    its d.  -> (banks {d: list of [T,d]}, queries list of (d, [T,d]))."""
    rc = np.random.default_rng(1000 + seed)
    banks = {}
    for D in dims:
        banks[D] = [_f32(znorm(correlated_walks(rc, 1, int(rc.integers(tmin, tmax + 1)), D))[0])
                    for _ in range(nc_per_bank)]
    rq = np.random.default_rng(2000 + seed)
    queries = []
    for _ in range(nq):
        D = int(rq.choice(dims))
        m = int(rq.integers(tmin, tmax + 1))
        queries.append((D, _f32(znorm(correlated_walks(rq, 1, m, D))[0])))
    return banks, queries


def loss_pairs(npairs=256, T=512, D=12, seed=5, jitter=1e-3):
    """Differentiable-DTW workload: independent random walks plus i.i.d.
    N(0, jitter^2) noise (breaks ties), not normalised.
    Full size: 256 pairs, length 512, d = 12, window 10%."""
    rng = np.random.default_rng(3000 + seed)
    x = random_walks(rng, npairs, T, D) + jitter * rng.standard_normal((npairs, T, D))
    y = random_walks(rng, npairs, T, D) + jitter * rng.standard_normal((npairs, T, D))
    return _f32(x), _f32(y)
