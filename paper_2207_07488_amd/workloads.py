"""Seeded synthetic inputs shared by the library's users, its tests and the oracle's tests.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic. Everything derives from SplitMix64 (Steele, Lea, Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014): output i of the
stream with seed s is mix(s + (i + 1) * 0x9E3779B97F4A7C15), and a double in
[0, 1) is (output >> 11) * 2**-53.

Workloads (the paper's networks are not published; Sec. 6.1 describes the
generator, whose parameters the caller chooses):

* fiber segments: straight segments of fixed length with uniform random
  midpoints and uniform random directions (angle in 2D, sphere in 3D, drawn
  by rejection from the cube so that no trigonometry is needed);
* grid network of Example 3.7 (nodes (i/n, j/n), edges of length 1/n);
* right-hand sides, i.i.d. uniform per free dof;
* Poisson arrival times for the serving mix.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_DIR_STREAM = 0x632BE59BD9B4E019  # offset of the direction stream from the midpoint stream


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start .. start+count-1 of the SplitMix64 stream seeded with `seed`."""
    i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, start: int, count: int) -> np.ndarray:
    """Doubles in [0, 1) from the stream, 53 random bits each."""
    return (splitmix64(seed, start, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def unit_directions(dim: int, n: int, seed: int) -> np.ndarray:
    """n directions uniform on the circle / sphere: candidates a in [-1, 1)^dim are
    accepted when 0 < |a|^2 <= 1 and normalised; acceptance is in stream order."""
    out = np.empty((0, dim))
    start = 0
    while out.shape[0] < n:
        need = n - out.shape[0]
        batch = max(64, int(need * (2.2 if dim == 3 else 1.4)) + 16)
        a = 2.0 * uniform01(seed, start, batch * dim).reshape(batch, dim) - 1.0
        start += batch * dim
        r2 = np.zeros(batch)
        for k in range(dim):
            r2 = r2 + a[:, k] * a[:, k]
        ok = (r2 > 0.0) & (r2 <= 1.0)
        a = a[ok] / np.sqrt(r2[ok])[:, None]
        out = np.concatenate([out, a], axis=0)
    return np.ascontiguousarray(out[:n])


def fiber_segments(dim: int, n_segments: int, length: float, seed: int,
                   margin: float = 0.0) -> np.ndarray:
    """Raw (unclipped) fiber segments, shape (n, 2*dim): [a_0..a_{d-1}, b_0..b_{d-1}].

    Midpoints are uniform in [-margin, 1 + margin]^dim (margin 0: the unit box;
    Sec. 6.1 uses margin 0.5*length)."""
    m = uniform01(seed, 0, n_segments * dim).reshape(n_segments, dim)
    m = -margin + m * (1.0 + 2.0 * margin)
    t = unit_directions(dim, n_segments, (seed + _DIR_STREAM) & 0xFFFFFFFFFFFFFFFF)
    half = 0.5 * length
    seg = np.empty((n_segments, 2 * dim))
    seg[:, :dim] = m - half * t
    seg[:, dim:] = m + half * t
    return np.ascontiguousarray(seg)


def rhs(n: int, k: int, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Right-hand sides, shape (n, k) (dof-major), column j i.i.d. uniform[lo, hi)
    from the stream seeded with seed + (j + 1) * 2**32."""
    f = np.empty((n, k))
    for j in range(k):
        f[:, j] = lo + (hi - lo) * uniform01((seed + (j + 1) * (1 << 32)) & 0xFFFFFFFFFFFFFFFF, 0, n)
    return f


def grid_network(n: int):
    """Grid network of Example 3.7: nodes (i/n, j/n), i fastest, edges between
    nodes at distance 1/n. Returns (coords (N,2), edges (E,2) int32)."""
    i = np.arange(n + 1, dtype=np.float64)
    X, Y = np.meshgrid(i / n, i / n, indexing="xy")
    coords = np.stack([X.ravel(), Y.ravel()], axis=1)
    idx = np.arange((n + 1) * (n + 1)).reshape(n + 1, n + 1)
    h = np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], axis=1)
    v = np.stack([idx[:-1, :].ravel(), idx[1:, :].ravel()], axis=1)
    edges = np.concatenate([h, v], axis=0).astype(np.int32)
    return np.ascontiguousarray(coords), np.ascontiguousarray(edges)


def boundary_flags(coords: np.ndarray, dir_lo: int, dir_hi: int, band: float) -> np.ndarray:
    """Dirichlet flags for a network given as arrays: within `band` of a Gamma face."""
    d = np.zeros(coords.shape[0], dtype=np.uint8)
    for k in range(coords.shape[1]):
        if (dir_lo >> k) & 1:
            d |= (coords[:, k] <= band).astype(np.uint8)
        if (dir_hi >> k) & 1:
            d |= (coords[:, k] >= 1.0 - band).astype(np.uint8)
    return d


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """n arrival times of a Poisson process with the given rate (per second)."""
    u = uniform01(seed, 0, n)
    gaps = -np.log1p(-u) / rate
    return np.cumsum(gaps)


# Workload presets. Sizes and parameters of the benchmark configurations.
# 2D: Dirichlet on x = 0 and x = 1 (axis 0, both faces); 3D: z = 0 and z = 1.
PRESETS = {
    "fiber2d_300": dict(dim=2, n_segments=300, length=0.2, seed=1, dir_lo=1, dir_hi=1, nH=4),
    "fiber2d_20k": dict(dim=2, n_segments=20000, length=0.05, seed=2, dir_lo=1, dir_hi=1, nH=32),
    "fiber3d_100k": dict(dim=3, n_segments=100000, length=0.05, seed=3, dir_lo=4, dir_hi=4, nH=16,
                         contact_eps=0.005),
    "truss3d_30k": dict(dim=3, n_segments=30000, length=0.1, seed=4, dir_lo=4, dir_hi=0, nH=16,
                        contact_eps=0.005, model=1),
}
BAND = 1e-3


def merge_tol(length: float) -> float:
    """Merge distance of Sec. 6.1: fiber length times 1e-4."""
    return length * 1e-4


def serving_pool(count: int, seed: int, n_min: float = 2e3, n_max: float = 5e5) -> list:
    """Networks of a serving mix: node counts log-uniform in [n_min, n_max],
    2D and 3D alternating, fiber density well above percolation, and the mesh
    chosen so that stars hold about 500 nodes on average.

    2D: segments n = N / (2 + D/pi) at density n l^2 = D = 20 (about D/pi
    crossings per segment). 3D: n = N / 4 with l = (25.5/n)^(1/3) and contact
    distance l/10 (about 4 contacts per segment). Mesh: 4N/nH^2 = 500 (2D),
    8N/nH^3 = 500 (3D), the 3D coarse space capped below 8192 dofs.
    """
    u = uniform01(seed, 0, count)
    out = []
    for i in range(count):
        N = float(np.exp(np.log(n_min) + (np.log(n_max) - np.log(n_min)) * u[i]))
        if i % 2 == 0:
            D = 20.0
            n = max(int(N / (2.0 + D / np.pi)), 16)
            length = float(np.sqrt(D / n))
            nH = max(2, int(round(np.sqrt(4.0 * N / 500.0))))
            out.append(dict(dim=2, n_segments=n, length=length, seed=seed * 1000 + i, dir_lo=1, dir_hi=1, nH=nH,
                            target_nodes=int(N)))
        else:
            n = max(int(N / 4.0), 16)
            length = float((25.5 / n) ** (1.0 / 3.0))
            nH = min(19, max(2, int(round((8.0 * N / 500.0) ** (1.0 / 3.0)))))
            out.append(dict(dim=3, n_segments=n, length=length, contact_eps=length / 10.0, seed=seed * 1000 + i,
                            dir_lo=4, dir_hi=4, nH=nH, target_nodes=int(N)))
    return out

