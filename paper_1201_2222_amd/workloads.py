"""Seeded synthetic inputs shared by the HIP path's tests, the benchmark and the
oracle tests.

This module only draws fields (opacity, destruction probability, thermal source
function, frequency weights) with the shapes, value distributions and boundary
layout of the workloads below; it holds none of the radiative transfer arithmetic.
Arrays are FP64, layout [nf][nz][ny][nx] (x fastest), unit cell spacing, k = 0 the
bottom.  Boundaries: periodic x and y, thermal bottom, vacuum top.  Dimensionless
units with sigma_B/pi = 1 (grey B = T^4) and 2h/c^2 = 1 (B_nu = x^3/(e^(x/T) - 1),
x = h nu / k T_ref).

Workloads (grid, rays, physics):
  plain      32^3, grey LTE pure absorber (eps = 1), chi lognormal(0, 1) per cell
             scaled to a mean vertical tau of 10, T ~ U[0.5, 1.5], 24 rays.
  scattering 128^3, grey, chi exponentially stratified (scale height 16 cells,
             vertical tau 1e4 at the bottom), eps = 1e-3, T = 1 + 0.2 g/max|g| for a
             sum g of 8 random Fourier modes, 48 rays.
  multifreq  192^3 x 64 log-spaced bins in x = [0.05, 50], chi_abs = kappa0 x^-3 rho
             with rho lognormal(0, 0.8), grey electron scattering with vertical tau
             10, Planck B_nu with T lognormal(0, 0.3), 80 rays.
  batched    one of many uneven problems solved together (seed 1004 + index): each
             axis 24..96 cells, 24/48/80 rays, 1..16 bins, eps = 10^U[-4, 0], grey
             chi lognormal(0, 1) scaled to a vertical tau of 10, T ~ U[0.5, 1.5],
             B = T^4 for one bin, else Planck bins on x = [0.05, 50].
  serving    request problems (seed 1005 + index): cubic N log-uniform in [32, 160],
             8..32 Planck bins, 48 rays, eps = 10^U[-4, 0], chi and T as batched;
             drifting snapshot streams scale T by 1 + 0.02 h with h a smooth 8-mode
             field (max |h| = 1) per step.  serving_request draws the same recipe
             with its per-cell fields generated on the device (one new problem per
             request of the serving benchmark).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

VACUUM, THERMAL, PERIODIC, FIXED = 0, 1, 2, 3


@dataclass
class Workload:
    name: str
    shape: tuple            # (nx, ny, nz)
    n_mu: int
    chi: np.ndarray         # [nf][nz][ny][nx]
    eps: np.ndarray
    B: np.ndarray
    w_nu: np.ndarray        # [nf]
    delta_c: float = 1e-6
    bc_lo: tuple = (PERIODIC, PERIODIC, THERMAL)
    bc_hi: tuple = (PERIODIC, PERIODIC, VACUUM)
    h: tuple = (1.0, 1.0, 1.0)
    meta: dict = field(default_factory=dict)

    @property
    def nf(self):
        return self.chi.shape[0]

    @property
    def na(self):
        return self.n_mu * (self.n_mu + 2)

    @property
    def cells(self):
        return int(np.prod(self.shape))


def _fields(nf, shape):
    nx, ny, nz = shape
    return (nf, nz, ny, nx)


def plain(n=32, seed=1001, n_mu=4):
    """Grey LTE pure absorber (eps = 1, S = B): one formal solution plus J, H, K."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    chi = np.exp(rng.normal(0.0, 1.0, _fields(1, shape)))
    chi *= 10.0 / chi.sum(axis=1).mean()           # mean vertical optical depth 10
    T = rng.uniform(0.5, 1.5, _fields(1, shape))
    B = T ** 4
    eps = np.ones_like(chi)
    return Workload("plain", shape, n_mu, chi, eps, B, np.ones(1), delta_c=1e-12)


def _fourier_field(rng, shape, modes=8, kmax=4):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    g = np.zeros((nz, ny, nx))
    for _ in range(modes):
        while True:
            kv = rng.integers(-kmax, kmax + 1, 3)
            if np.any(kv != 0):
                break
        a = rng.uniform(0.5, 1.0)
        phi = rng.uniform(0.0, 2.0 * np.pi)
        g += a * np.cos(2.0 * np.pi * (kv[0] * x / nx + kv[1] * y / ny + kv[2] * z / nz) + phi)
    return g / np.max(np.abs(g))


def scattering(n=128, seed=1002, n_mu=6, eps=1e-3, tau_bottom=1e4, scale_height=None):
    """Grey coherent scattering atmosphere, Jacobi ALI to max |dS/S| < 1e-6.  For
    n != 128 the scale height is scaled with n (16 cells at n = 128)."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    hs = 16.0 * n / 128.0 if scale_height is None else scale_height
    k = np.arange(n)
    prof = np.exp(-k / hs)
    prof *= tau_bottom / prof.sum()
    chi = np.broadcast_to(prof[None, :, None, None], _fields(1, shape)).copy()
    T = 1.0 + 0.2 * _fourier_field(rng, shape)
    B = (T ** 4)[None]
    epsa = np.full(_fields(1, shape), eps)
    return Workload("scattering", shape, n_mu, chi, epsa, B, np.ones(1), delta_c=1e-6,
                    meta={"eps": eps, "tau_bottom": tau_bottom, "scale_height": hs})


def multifreq(n=192, nf=64, seed=1003, n_mu=8, bins=None):
    """Multi-frequency free-free + electron scattering atmosphere.  ``bins`` selects
    a subset of the nf bins (bins are independent); the full grid of x_nu and w_nu
    is always built from nf."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    x = np.logspace(np.log10(0.05), np.log10(50.0), nf)
    w = np.zeros(nf)
    w[1:] += 0.5 * np.diff(x)
    w[:-1] += 0.5 * np.diff(x)
    rho = np.exp(rng.normal(0.0, 0.8, (n, n, n)))
    T = np.exp(rng.normal(0.0, 0.3, (n, n, n)))
    kappa0 = 10.0 / rho.sum(axis=0).mean()          # mean vertical absorption tau 10 at x = 1
    chi_sc = 10.0 / n
    sel = np.arange(nf) if bins is None else np.asarray(bins)
    chi = np.empty((len(sel), n, n, n))
    eps = np.empty_like(chi)
    B = np.empty_like(chi)
    for o, b in enumerate(sel):
        ca = kappa0 * x[b] ** -3 * rho
        chi[o] = ca + chi_sc
        eps[o] = ca / (ca + chi_sc)
        B[o] = x[b] ** 3 / np.expm1(x[b] / T)
    return Workload("multifreq", shape, n_mu, chi, eps, B, w[sel], delta_c=1e-6,
                    meta={"x_nu": x[sel], "bins": sel.tolist(), "nf_total": nf})


def random_problem(shape, nf=1, seed=0, n_mu=4, eps_range=(1e-2, 1.0), chi_sigma=1.0,
                   tau=10.0, bc_lo=(PERIODIC, PERIODIC, THERMAL), bc_hi=(PERIODIC, PERIODIC, VACUUM),
                   h=(1.0, 1.0, 1.0)):
    """Small random problem for parity tests: lognormal chi scaled to a vertical tau,
    log-uniform eps, B from T ~ U[0.5, 1.5]."""
    rng = np.random.default_rng(seed)
    fs = _fields(nf, shape)
    chi = np.exp(rng.normal(0.0, chi_sigma, fs))
    chi *= tau / (chi.sum(axis=1).mean() * h[2])
    lo, hi = np.log10(eps_range[0]), np.log10(eps_range[1])
    eps = 10.0 ** rng.uniform(lo, hi, fs)
    B = rng.uniform(0.5, 1.5, fs) ** 4
    return Workload("random", tuple(shape), n_mu, chi, eps, B, rng.uniform(0.5, 1.5, nf),
                    bc_lo=tuple(bc_lo), bc_hi=tuple(bc_hi), h=tuple(h))


def _planck_bins(nf, T):
    x = np.logspace(np.log10(0.05), np.log10(50.0), nf)
    w = np.zeros(nf)
    w[1:] += 0.5 * np.diff(x)
    w[:-1] += 0.5 * np.diff(x)
    B = np.stack([x[b] ** 3 / np.expm1(x[b] / T) for b in range(nf)])
    return B, w


def batched_problem(index, seed=1004, min_n=24, max_n=96):
    """Problem ``index`` of the uneven batch (sizes, rays, bins and eps drawn per problem)."""
    rng = np.random.default_rng(seed + index)
    nx, ny, nz = (int(v) for v in rng.integers(min_n, max_n + 1, 3))
    n_mu = int(rng.choice([4, 6, 8]))
    nf = int(rng.integers(1, 17))
    eps = float(10.0 ** rng.uniform(-4.0, 0.0))
    shape = (nx, ny, nz)
    chi1 = np.exp(rng.normal(0.0, 1.0, (nz, ny, nx)))
    chi1 *= 10.0 / chi1.sum(axis=0).mean()
    T = rng.uniform(0.5, 1.5, (nz, ny, nx))
    if nf == 1:
        B = (T ** 4)[None]
        w = np.ones(1)
    else:
        B, w = _planck_bins(nf, T)
    chi = np.broadcast_to(chi1[None], B.shape).copy()
    epsa = np.full(B.shape, eps)
    return Workload("batched", shape, n_mu, chi, epsa, B, w, delta_c=1e-6, meta={"eps": eps, "index": index})


def serving_problem(index, seed=1005, min_n=32, max_n=160):
    """One request problem of the serving workload."""
    rng = np.random.default_rng(seed + index)
    n = int(round(np.exp(rng.uniform(np.log(min_n), np.log(max_n)))))
    nf = int(rng.integers(8, 33))
    eps = float(10.0 ** rng.uniform(-4.0, 0.0))
    shape = (n, n, n)
    chi1 = np.exp(rng.normal(0.0, 1.0, (n, n, n)))
    chi1 *= 10.0 / chi1.sum(axis=0).mean()
    T = rng.uniform(0.5, 1.5, (n, n, n))
    B, w = _planck_bins(nf, T)
    chi = np.broadcast_to(chi1[None], B.shape).copy()
    epsa = np.full(B.shape, eps)
    return Workload("serving", shape, 6, chi, epsa, B, w, delta_c=1e-6,
                    meta={"eps": eps, "index": index, "T": T})


def drift(T, step, seed=1005):
    """Next snapshot of a drifting stream: T (1 + 0.02 h) with a smooth 8-mode field h
    drawn for this step (max |h| = 1)."""
    rng = np.random.default_rng(seed * 1000 + step)
    nz, ny, nx = T.shape
    h = _fourier_field(rng, (nx, ny, nz))
    return T * (1.0 + 0.02 * h)


# ---- serving requests generated on the device ---------------------------------------
# The serving workload draws a new problem for every request (thousands per run), so its
# fields are drawn with torch on the device: the request's scalars (grid edge, bins,
# eps) from numpy with the request's seed, the per-cell fields from a torch generator
# seeded from it.  The arrays follow serving_problem's recipe.

def _torch_planck(x, T):
    import torch
    return x ** 3 / torch.expm1(x / T)


def _torch_fourier(gen, n, device, modes=8, kmax=4):
    """Smooth field of 8 random Fourier modes on an n^3 grid, max |h| = 1."""
    import torch
    ax = torch.arange(n, device=device, dtype=torch.float64)
    z, y, x = torch.meshgrid(ax, ax, ax, indexing="ij")
    g = torch.zeros((n, n, n), dtype=torch.float64, device=device)
    for _ in range(modes):
        while True:
            kv = torch.randint(-kmax, kmax + 1, (3,), generator=gen, device=device)
            if bool((kv != 0).any()):
                break
        a = 0.5 + 0.5 * torch.rand((), generator=gen, device=device, dtype=torch.float64)
        phi = 2.0 * np.pi * torch.rand((), generator=gen, device=device, dtype=torch.float64)
        g += a * torch.cos(2.0 * np.pi * (kv[0] * x + kv[1] * y + kv[2] * z) / n + phi)
    return g / g.abs().max()


def serving_request(index, device="cuda", seed=1005, min_n=32, max_n=160, n=None, nf=None):
    """Request ``index`` of the serving workload with its fields on ``device``: cubic N
    log-uniform in [32, 160] (or ``n``), 8..32 Planck bins (or ``nf``), 48 rays, eps =
    10^U[-4, 0], grey chi lognormal(0, 1) scaled to a vertical tau of 10, T ~
    U[0.5, 1.5].  Returns a dict of flat device tensors chi, eps, B ([nf][n^3]), the
    frequency weights and T ([n^3]) for drifting streams."""
    import torch
    rng = np.random.default_rng(seed + 7919 * index)
    n_ = int(round(np.exp(rng.uniform(np.log(min_n), np.log(max_n))))) if n is None else int(n)
    nf_ = int(rng.integers(8, 33)) if nf is None else int(nf)
    eps = float(10.0 ** rng.uniform(-4.0, 0.0))
    gen = torch.Generator(device=device)
    gen.manual_seed(int(rng.integers(0, 2 ** 62)))
    chi1 = torch.exp(torch.randn((n_, n_, n_), generator=gen, device=device, dtype=torch.float64))
    chi1 *= 10.0 / chi1.sum(dim=0).mean()
    T = 0.5 + torch.rand((n_, n_, n_), generator=gen, device=device, dtype=torch.float64)
    x = np.logspace(np.log10(0.05), np.log10(50.0), nf_)
    w = np.zeros(nf_)
    w[1:] += 0.5 * np.diff(x)
    w[:-1] += 0.5 * np.diff(x)
    B = torch.stack([_torch_planck(float(xb), T) for xb in x]).reshape(-1)
    chi = chi1.reshape(1, -1).expand(nf_, -1).reshape(-1).contiguous()
    return {"shape": (n_, n_, n_), "nf": nf_, "n_mu": 6, "eps_value": eps, "chi": chi,
            "eps": torch.full_like(chi, eps), "B": B, "w_nu": w, "x_nu": x, "T": T.reshape(-1), "gen": gen}


def serving_drift(req, step, device="cuda", seed=1005):
    """Next snapshot of a drifting stream: T (1 + 0.02 h) with a smooth 8-mode field h
    drawn for this step (max |h| = 1); returns the new B (the stream's chi and eps stay)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed * 1000003 + 101 * step + req["shape"][0])
    n = req["shape"][0]
    h = _torch_fourier(gen, n, device).reshape(-1)
    req["T"] = req["T"] * (1.0 + 0.02 * h)
    req["B"] = torch.stack([_torch_planck(float(xb), req["T"]) for xb in req["x_nu"]]).reshape(-1)
    return req["B"]
