"""Seeded synthetic workloads shaped like the paper's experiments.

The paper measures on UCI data sets (Table 1) that are not available here; these
generators stand in for them.  Every workload is a mixture of isotropic Gaussian
blobs plus uniform noise in the unit hypercube, quantised to int32 fixed point
(``floor(x * 2**q + 0.5)``) so that every squared distance is an exact integer.

This module holds no clustering arithmetic: it only draws inputs.  Both the GPU
path and the CPU oracle consume what it returns.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = ["Workload", "make_blobs", "make_config", "CONFIG_NAMES", "quantise"]


@dataclass
class Workload:
    """One clustering job: int32 fixed-point points plus the DBSCAN parameters."""

    name: str
    points: np.ndarray          # int32 [n, d], row-major, fixed-point units
    eps: float                  # radius in the same fixed-point units (eps_real * 2**q)
    min_pts: int
    q: int                      # fixed-point fraction bits
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    @property
    def d(self) -> int:
        return int(self.points.shape[1])


def quantise(x: np.ndarray, q: int) -> np.ndarray:
    """Round real coordinates to int32 multiples of 2**-q (round half up)."""
    y = np.floor(np.asarray(x, dtype=np.float64) * float(2 ** q) + 0.5)
    if y.size and (y.max() > np.iinfo(np.int32).max or y.min() < np.iinfo(np.int32).min):
        raise OverflowError("quantised coordinates do not fit in int32")
    return y.astype(np.int32)


def make_blobs(rng: np.random.Generator, n: int, d: int, n_blobs: int, stds,
               noise_frac: float, sizes: str = "equal") -> np.ndarray:
    """Real-valued points: ``n_blobs`` Gaussian blobs (centres uniform in [0,1]^d)
    plus ``round(noise_frac * n)`` uniform noise points, in one random order.

    ``stds`` is a scalar or one standard deviation per blob.  ``sizes`` is
    ``"equal"`` (multinomial with equal shares) or ``"dirichlet"`` (shares drawn
    from Dirichlet(1, ..., 1), then multinomial)."""
    n_noise = int(round(noise_frac * n))
    n_blob = n - n_noise
    centres = rng.uniform(0.0, 1.0, size=(n_blobs, d))
    stds = np.broadcast_to(np.asarray(stds, dtype=np.float64), (n_blobs,))
    if sizes == "equal":
        shares = np.full(n_blobs, 1.0 / n_blobs)
    elif sizes == "dirichlet":
        shares = rng.dirichlet(np.ones(n_blobs))
    else:
        raise ValueError(f"unknown sizes mode {sizes!r}")
    counts = rng.multinomial(n_blob, shares)
    parts = [centres[b] + stds[b] * rng.standard_normal(size=(int(counts[b]), d))
             for b in range(n_blobs)]
    parts.append(rng.uniform(0.0, 1.0, size=(n_noise, d)))
    x = np.concatenate(parts, axis=0) if parts else np.zeros((0, d))
    perm = rng.permutation(x.shape[0])
    return x[perm]


def _cfg_small(seed: int) -> Workload:
    # 2-D, 10,000 points: five blobs (std 0.03), 5 % noise, 2^-12 units.
    rng = np.random.Generator(np.random.PCG64(seed))
    q = 12
    x = make_blobs(rng, 10_000, 2, 5, 0.03, 0.05, "equal")
    return Workload("blobs2d_10k", quantise(x, q), 0.02 * 2 ** q, 4, q,
                    {"eps_real": 0.02, "seed": seed})


def _cfg_2d_1m(seed: int, n: int = 1_000_000) -> Workload:
    # 2-D, 1M points: 50 blobs, std log-uniform in [0.002, 0.01], Dirichlet(1)
    # sizes, 10 % noise, 2^-16 units.
    rng = np.random.Generator(np.random.PCG64(seed))
    q = 16
    stds = np.exp(rng.uniform(np.log(0.002), np.log(0.01), size=50))
    x = make_blobs(rng, n, 2, 50, stds, 0.10, "dirichlet")
    return Workload("blobs2d_1m" if n == 1_000_000 else f"blobs2d_{n}", quantise(x, q),
                    0.004 * 2 ** q, 8, q, {"eps_real": 0.004, "seed": seed})


def _cfg_8d_500k(seed: int, n: int = 500_000) -> Workload:
    # 8-D, 500k points: 20 blobs (std 0.02), 5 % noise, 2^-12 units.
    rng = np.random.Generator(np.random.PCG64(seed))
    q = 12
    x = make_blobs(rng, n, 8, 20, 0.02, 0.05, "equal")
    return Workload("blobs8d_500k" if n == 500_000 else f"blobs8d_{n}", quantise(x, q),
                    0.06 * 2 ** q, 10, q, {"eps_real": 0.06, "seed": seed})


def make_high(d: int, n: int, seed: int = 6) -> Workload:
    """Data with many axes, built like the 8-D workload: 20 blobs (std 0.02),
    5 % noise, 2^-12 units, minPts 10, and eps = 0.015 * sqrt(2 d) (0.06 at
    d = 8: three quarters of the typical distance between two points of a
    blob).  At d = 54 and n = 3,850,505 it has the shape of the paper's
    largest data set (PAMAP2, Table 1)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, d, n])))
    q = 12
    eps = 0.015 * float(np.sqrt(2.0 * d))
    x = make_blobs(rng, n, d, 20, 0.02, 0.05, "equal")
    return Workload(f"blobs{d}d_{n}", quantise(x, q), eps * 2 ** q, 10, q,
                    {"eps_real": eps, "seed": seed})


def make_mixed(seed: int, n: int, d: int, q: int = 14) -> Workload:
    """One job of the mixed-size family: 3-30 blobs with per-blob std uniform in
    [0.005, 0.03], 5-15 % noise, eps uniform in [0.005, 0.03], minPts in 4..12."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_blobs = int(rng.integers(3, 31))
    stds = rng.uniform(0.005, 0.03, size=n_blobs)
    noise = float(rng.uniform(0.05, 0.15))
    eps = float(rng.uniform(0.005, 0.03))
    min_pts = int(rng.integers(4, 13))
    x = make_blobs(rng, n, d, n_blobs, stds, noise, "equal")
    return Workload(f"mixed{d}d_{n}", quantise(x, q), eps * 2 ** q, min_pts, q,
                    {"eps_real": eps, "seed": seed, "blobs": n_blobs, "noise": noise})


def make_batch(seed: int = 4, count: int = 256, n_range=(1_000, 200_000), dims=(2, 3, 4),
               q: int = 14) -> list:
    """The batched workload: ``count`` independent jobs, job k drawn from the
    k-th child of ``SeedSequence(seed)``.  Each job has n log-uniform in
    ``n_range``, d uniform in ``dims``, 3-30 blobs with per-blob std uniform in
    [0.005, 0.03] (multinomial sizes, equal shares), 5-15 % noise, eps uniform
    in [0.005, 0.03] and minPts uniform in 4..12; coordinates are 2^-q fixed
    point."""
    jobs = []
    for k, child in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.Generator(np.random.PCG64(child))
        n = int(round(float(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]))))))
        d = int(rng.choice(np.asarray(dims)))
        n_blobs = int(rng.integers(3, 31))
        stds = rng.uniform(0.005, 0.03, size=n_blobs)
        noise = float(rng.uniform(0.05, 0.15))
        eps = float(rng.uniform(0.005, 0.03))
        min_pts = int(rng.integers(4, 13))
        x = make_blobs(rng, n, d, n_blobs, stds, noise, "equal")
        jobs.append(Workload(f"batch{seed}_{k}_{d}d_{n}", quantise(x, q), eps * 2 ** q, min_pts, q,
                             {"eps_real": eps, "seed": seed, "job": k, "blobs": n_blobs, "noise": noise}))
    return jobs


def make_served(seed: int = 5, count: int = 64, n_range=(10_000, 2_000_000), dims=(2, 3, 5),
                q: int = 14) -> list:
    """Request data sets of the served workload: job k drawn from the k-th
    child of ``SeedSequence(seed)``, with the batched workload's recipe but n
    log-uniform in ``n_range`` and d uniform in ``dims``."""
    return make_batch(seed=seed, count=count, n_range=n_range, dims=dims, q=q)


def served_requests(seed: int = 5, count: int = 10_000, n_range=(10_000, 2_000_000), dims=(2, 3, 5),
                    q: int = 14) -> list:
    """Parameters of ``count`` distinct requests of the served workload (the
    batched workload's recipe: 3-30 blobs with per-blob std uniform in
    [0.005, 0.03], 5-15 % noise, eps uniform in [0.005, 0.03], minPts in
    4..12; n log-uniform in ``n_range``, d uniform in ``dims``), drawn on the
    host; the points themselves come from :func:`device_request`."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 2])))
    out = []
    for k in range(count):
        n = int(round(float(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]))))))
        d = int(rng.choice(np.asarray(dims)))
        n_blobs = int(rng.integers(3, 31))
        out.append({"k": k, "seed": seed, "n": n, "d": d, "q": q,
                    "centres": rng.uniform(0.0, 1.0, size=(n_blobs, d)),
                    "stds": rng.uniform(0.005, 0.03, size=n_blobs),
                    "noise": float(rng.uniform(0.05, 0.15)),
                    "eps": float(rng.uniform(0.005, 0.03)) * 2 ** q,
                    "min_pts": int(rng.integers(4, 13))})
    return out


def device_request(req: dict, device):
    """The points of one served request, drawn on the device by a torch
    generator seeded from (seed, k): each blob point takes a blob uniformly
    (equal shares), a Gaussian offset of that blob's std around its centre,
    then the noise points uniform in [0,1]^d, one random order, quantised to
    int32 as floor(x * 2^q + 0.5)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(req["seed"]) * 1_000_003 + int(req["k"]))
    n, d = int(req["n"]), int(req["d"])
    n_noise = int(round(req["noise"] * n))
    centres = torch.as_tensor(req["centres"], dtype=torch.float64, device=device)
    stds = torch.as_tensor(req["stds"], dtype=torch.float64, device=device)
    which = torch.randint(0, centres.shape[0], (n - n_noise,), generator=g, device=device)
    blob = centres[which] + stds[which, None] * torch.randn(n - n_noise, d, generator=g, device=device,
                                                               dtype=torch.float64)
    noise = torch.rand(n_noise, d, generator=g, device=device, dtype=torch.float64)
    x = torch.cat([blob, noise])[torch.randperm(n, generator=g, device=device)]
    return torch.floor(x * float(2 ** req["q"]) + 0.5).to(torch.int32).contiguous()


def poisson_arrivals(seed: int, count: int, rate: float) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 1])))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


CONFIG_NAMES = {1: "blobs2d_10k", 2: "blobs2d_1m", 3: "blobs8d_500k"}


def make_config(k: int, seed: int | None = None, n: int | None = None) -> Workload:
    """The fixed workloads: 1 = 2-D 10k, 2 = 2-D 1M, 3 = 8-D 500k.

    ``seed`` defaults to ``k``; ``n`` overrides the point count (same recipe)."""
    seed = k if seed is None else seed
    if k == 1:
        return _cfg_small(seed)
    if k == 2:
        return _cfg_2d_1m(seed, n or 1_000_000)
    if k == 3:
        return _cfg_8d_500k(seed, n or 500_000)
    raise ValueError(f"unknown workload {k}")
