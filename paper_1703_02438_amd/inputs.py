"""Seeded synthetic snapshot generators.

This module only makes input data: pairs of consecutive snapshots of a
simulation variable, shaped like the workloads the NUMARCK paper compresses
(FLASH turbulence and Sedov fields, ASR/CMIP climate grids; Table 1).  None of
the paper's datasets are available, so each generator states its recipe.  It
holds none of the compression method's arithmetic and is shared by the tests,
the benchmark and the serving driver.

All generators are deterministic for a given seed and device.  They use torch
so that the large workloads can be generated directly in device memory; on the
CPU they are used for the small test cases.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def mixture_ratios(n: int, g: torch.Generator, device, dtype=torch.float64) -> torch.Tensor:
    """Per-point relative change drawn from a 3-component mixture:
    70 % N(0, 0.002), 25 % N(0.01, 0.005), 5 % U[-0.5, 0.5]."""
    u = torch.rand(n, generator=g, device=device, dtype=dtype)
    a = torch.randn(n, generator=g, device=device, dtype=dtype) * 0.002
    b = torch.randn(n, generator=g, device=device, dtype=dtype) * 0.005 + 0.01
    c = torch.rand(n, generator=g, device=device, dtype=dtype) - 0.5
    return torch.where(u < 0.70, a, torch.where(u < 0.95, b, c))


def lognormal_field(n: int, g: torch.Generator, device, zero_frac: float = 0.001,
                    dtype=torch.float64) -> torch.Tensor:
    """x ~ lognormal(0, 1) with exactly round(zero_frac * n) entries set to 0."""
    x = torch.exp(torch.randn(n, generator=g, device=device, dtype=dtype))
    nz = int(round(zero_frac * n))
    if nz:
        pos = torch.randperm(n, generator=g, device=device)[:nz]
        x[pos] = 0
    return x


def mixture_pair(n: int, seed: int, dtype=torch.float64, device="cpu"):
    """Plain single-variable workload (the 64^3 fp64 case and the per-variable
    data of the batched workload): prev ~ lognormal(0,1) with 0.1 % zeros,
    curr = prev * (1 + r) with r from :func:`mixture_ratios`.  For float32 the
    previous snapshot is rounded first and the product formed from it."""
    g = _gen(seed, device)
    prev64 = lognormal_field(n, g, device)
    r = mixture_ratios(n, g, device)
    if dtype == torch.float32:
        prev = prev64.to(torch.float32)
        curr = (prev.to(torch.float64) * (1 + r)).to(torch.float32)
        return prev, curr
    return prev64, prev64 * (1 + r)


def gaussian_smooth(x: torch.Tensor, sigma: float) -> torch.Tensor:
    """Periodic Gaussian smoothing (std sigma cells) of an N-d field via FFT,
    renormalised to zero mean and unit standard deviation."""
    dims = tuple(range(x.dim()))
    X = torch.fft.rfftn(x, dim=dims)
    k2 = None
    for ax, size in enumerate(x.shape):
        if ax == x.dim() - 1:
            f = torch.fft.rfftfreq(size, device=x.device, dtype=x.dtype)
        else:
            f = torch.fft.fftfreq(size, device=x.device, dtype=x.dtype)
        shape = [1] * x.dim()
        shape[ax] = -1
        f2 = (f * f).reshape(shape)
        k2 = f2 if k2 is None else k2 + f2
    X = X * torch.exp(-2.0 * math.pi ** 2 * sigma ** 2 * k2)
    y = torch.fft.irfftn(X, s=x.shape, dim=dims)
    y = y - y.mean()
    return y / y.std()


@dataclass
class FlashSeries:
    """FLASH-like 3-D turbulence series (stand-in for the Stir variables):
    x_0 = exp(G_4 * N(0,1)); x_{t+1} = x_t (1 + r_t) with
    r_t = 0.01 * (G_4 * N(0,1)) + Cauchy(0, 0.2) on a Bernoulli(0.02) mask,
    where G_4 * denotes periodic Gaussian smoothing with sigma = 4 cells
    followed by renormalisation to unit std.  float64."""
    edge: int = 512
    seed: int = 1705
    device: str = "cpu"
    sigma: float = 4.0
    shock_frac: float = 0.02
    shock_scale: float = 0.2
    amp: float = 0.01

    def __post_init__(self):
        self.g = _gen(self.seed, self.device)
        shape = (self.edge,) * 3
        w = torch.randn(shape, generator=self.g, device=self.device, dtype=torch.float64)
        self.x = torch.exp(gaussian_smooth(w, self.sigma)).reshape(-1)
        self.shape = shape

    def step(self) -> torch.Tensor:
        """Advance one snapshot; returns the new snapshot (flat float64)."""
        w = torch.randn(self.shape, generator=self.g, device=self.device, dtype=torch.float64)
        r = self.amp * gaussian_smooth(w, self.sigma).reshape(-1)
        del w
        u = torch.rand(r.numel(), generator=self.g, device=self.device, dtype=torch.float64)
        mask = torch.rand(r.numel(), generator=self.g, device=self.device,
                          dtype=torch.float64) < self.shock_frac
        shock = self.shock_scale * torch.tan(math.pi * (u - 0.5))
        r = r + torch.where(mask, shock, torch.zeros_like(shock))
        self.x = self.x * (1 + r)
        return self.x


@dataclass
class ClimateSeries:
    """Climate-like 2-D lat-lon series (stand-in for CMIP/ASR variables):
    nlat x nlon float32 grid, lat = -89.95 .. 89.95 degrees;
    x_0 = 250 + 30 cos(lat) + 5 (G_8 * N(0,1)); per step r ~ N(0, 3e-4) i.i.d.
    plus U[-a, a] added on 1 % of the cells (a = 0.05 by default);
    x_{t+1} = float32(float64(x_t) (1 + r))."""
    nlat: int = 1800
    nlon: int = 3600
    seed: int = 1707
    device: str = "cpu"
    sigma: float = 8.0
    noise: float = 3e-4
    outlier_frac: float = 0.01
    outlier_amp: float = 0.05
    outlier_lo: float | None = None
    outlier_hi: float | None = None

    def __post_init__(self):
        self.g = _gen(self.seed, self.device)
        lat = torch.linspace(-89.95, 89.95, self.nlat, device=self.device, dtype=torch.float64)
        w = torch.randn((self.nlat, self.nlon), generator=self.g, device=self.device,
                        dtype=torch.float64)
        base = 250 + 30 * torch.cos(torch.deg2rad(lat))[:, None] + 5 * gaussian_smooth(w, self.sigma)
        self.x = base.reshape(-1).to(torch.float32)

    def step(self) -> torch.Tensor:
        n = self.x.numel()
        r = torch.randn(n, generator=self.g, device=self.device, dtype=torch.float64) * self.noise
        m = torch.rand(n, generator=self.g, device=self.device, dtype=torch.float64) < self.outlier_frac
        lo = -self.outlier_amp if self.outlier_lo is None else self.outlier_lo
        hi = self.outlier_amp if self.outlier_hi is None else self.outlier_hi
        o = lo + (hi - lo) * torch.rand(n, generator=self.g, device=self.device, dtype=torch.float64)
        r = r + torch.where(m, o, torch.zeros_like(o))
        self.x = (self.x.to(torch.float64) * (1 + r)).to(torch.float32)
        return self.x


@dataclass
class VarSpec:
    edge: int
    dtype: torch.dtype
    E: float
    B: int
    seed: int

    @property
    def n(self) -> int:
        return self.edge ** 3


def batched_specs(count: int = 64, seed: int = 1706, lo_edge: int = 32, hi_edge: int = 384):
    """Uneven batched workload: cube edges log-uniform in [lo_edge, hi_edge],
    60 % float64 / 40 % float32, E from {1e-4, 1e-3, 1e-2}, B from {8, 10, 12}."""
    g = _gen(seed, "cpu")
    specs = []
    for i in range(count):
        u = torch.rand(4, generator=g, dtype=torch.float64).tolist()
        edge = int(round(math.exp(math.log(lo_edge) + u[0] * (math.log(hi_edge) - math.log(lo_edge)))))
        dt = torch.float64 if u[1] < 0.6 else torch.float32
        E = (1e-4, 1e-3, 1e-2)[min(int(u[2] * 3), 2)]
        B = (8, 10, 12)[min(int(u[3] * 3), 2)]
        specs.append(VarSpec(edge, dt, E, B, seed * 1000 + i))
    return specs


@dataclass
class ServeVar:
    n: int
    dtype: torch.dtype
    E: float
    B: int
    seed: int


def serving_specs(count: int = 32, seed: int = 1709, lo_bytes: int = 16 << 20,
                  hi_bytes: int = 4 << 30):
    """Live variables of the serving workload: sizes log-uniform in
    [lo_bytes, hi_bytes], float32 / float64 equally likely, E in {1e-4, 1e-3},
    B = 8."""
    g = _gen(seed, "cpu")
    out = []
    for i in range(count):
        u = torch.rand(3, generator=g, dtype=torch.float64).tolist()
        nbytes = math.exp(math.log(lo_bytes) + u[0] * (math.log(hi_bytes) - math.log(lo_bytes)))
        dt = torch.float32 if u[1] < 0.5 else torch.float64
        L = 4 if dt == torch.float32 else 8
        n = max(int(nbytes // L) // 4 * 4, 4)
        out.append(ServeVar(n, dt, (1e-4, 1e-3)[min(int(u[2] * 2), 1)], 8, seed * 1000 + i))
    return out


def serving_requests(specs, rate: float, count: int, range_frac: float = 0.05,
                     seed: int = 1710, range_fracs=(0.2, 0.4, 0.6, 0.8)):
    """`count` Poisson arrivals at `rate` per second: (time, var, kind, start,
    length); kind 0 = compress, 1 = range decompression of a contiguous range
    whose length is one of `range_fracs` of the variable (the partial
    decompressions of 20/40/60/80 % timed in the paper's Table 7), at a
    random start."""
    g = _gen(seed, "cpu")
    t, reqs = 0.0, []
    while len(reqs) < count:
        u = torch.rand(5, generator=g, dtype=torch.float64).tolist()
        t += -math.log(1.0 - u[0]) / rate
        v = min(int(u[1] * len(specs)), len(specs) - 1)
        n = specs[v].n
        if u[2] < range_frac:
            f = range_fracs[min(int(u[3] * len(range_fracs)), len(range_fracs) - 1)]
            ln = max(int(n * f), 1)
            st = min(int(u[4] * (n - ln + 1)), n - ln)
            reqs.append((t, v, 1, st, ln))
        else:
            reqs.append((t, v, 0, 0, 0))
    return reqs
