"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers; it holds none of the compressor's
arithmetic and is shared by the tests, the benchmark and the smoke check (both
the GPU path and the CPU oracle receive the same arrays from it).

The distributions stand in for the CTA Monte-Carlo files measured in the paper
(Sec. 4.3), which are not available: white Gaussian noise on a pedestal plus
sparse Cherenkov pulses (Sec. 2, Fig. 1), in camera-shaped events.
"""
from __future__ import annotations

import math

import numpy as np
import torch

PULSE_MEAN = 200.0  # mean pulse amplitude (exponential), ADC counts
PULSE_SIGMA_T = 1.0  # Gaussian pulse width in samples (so +-2 sigma spans 4 samples)

CAMERA_SHAPES = [(1855, 40), (2048, 96), (11328, 128)]


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def tiny_gaussian(n: int = 1 << 20, seed: int = 0, device="cpu") -> torch.Tensor:
    """round(N(300, 4^2)) clipped to [0, 65535], as uint16."""
    g = _gen(seed, device)
    x = torch.randn(n, generator=g, device=device, dtype=torch.float32) * 4.0 + 300.0
    return x.round_().clamp_(0, 65535).to(torch.int32).to(torch.uint16)


def _pulse_events(E: int, P: int, S: int, sigma, frac, pedestal: float, g, device, maxval: int,
                  out_dtype) -> torch.Tensor:
    """E events of P pixel traces of S samples: pedestal + round(N(0, sigma^2)) noise plus
    Gaussian-shaped pulses of amplitude Exp(mean 200) on round(frac * P) pixels per event
    (pixels drawn without replacement, pulse centre uniform over the trace)."""
    sig = torch.as_tensor(sigma, dtype=torch.float32, device=device).reshape(-1, 1, 1).expand(E, 1, 1)
    x = torch.randn(E, P, S, generator=g, device=device, dtype=torch.float32) * sig
    x = x.round_() + pedestal
    fr = torch.as_tensor(frac, dtype=torch.float32, device=device).reshape(-1).expand(E)
    npulse = torch.round(fr * P).to(torch.int64)
    kmax = int(npulse.max().item()) if E else 0
    if kmax > 0:
        order = torch.rand(E, P, generator=g, device=device).argsort(dim=1)[:, :kmax]
        amp = -torch.log1p(-torch.rand(E, kmax, generator=g, device=device)) * PULSE_MEAN
        t0 = torch.randint(0, S, (E, kmax), generator=g, device=device).to(torch.float32)
        keep = (torch.arange(kmax, device=device).reshape(1, -1) < npulse.reshape(-1, 1)).to(torch.float32)
        t = torch.arange(S, device=device, dtype=torch.float32).reshape(1, 1, S)
        shape = torch.exp(-0.5 * ((t - t0.unsqueeze(-1)) / PULSE_SIGMA_T) ** 2)
        pulses = (amp * keep).unsqueeze(-1) * shape
        x.scatter_add_(1, order.unsqueeze(-1).expand(E, kmax, S), pulses)
    x = x.round_().clamp_(0, maxval)
    if out_dtype == torch.uint16:
        return x.to(torch.int32).to(torch.uint16)
    return x.to(torch.int64).to(torch.uint32)


def camera_events(events: int, seed: int = 1, device="cpu", pixels: int = 1855, samples: int = 40,
                  sigma: float = 6.0, pulse_frac: float = 0.02, pedestal: float = 250.0,
                  chunk: int = 500) -> torch.Tensor:
    """Camera-shaped u16 waveforms [events, pixels, samples] (block = one pixel trace)."""
    out = torch.empty(events, pixels, samples, dtype=torch.uint16, device=device)
    g = _gen(seed, device)
    for e0 in range(0, events, chunk):
        e1 = min(events, e0 + chunk)
        out[e0:e1] = _pulse_events(e1 - e0, pixels, samples, sigma, pulse_frac, pedestal, g, device,
                                   65535, torch.uint16)
    return out


def uneven_events(events: int, seed: int = 3, device="cpu", shapes=None):
    """Batched uneven events: shape ~ U{1855x40, 2048x96, 11328x128}, dtype ~ U{u16, u32},
    noise sigma ~ U(2, 20), pulse fraction ~ U(0, 5%). Returns a list of 2-D tensors."""
    shapes = shapes or CAMERA_SHAPES
    rng = np.random.default_rng(seed)
    g = _gen(seed, device)
    out = []
    kinds = rng.integers(0, len(shapes), events)
    dts = rng.integers(0, 2, events)
    sig = rng.uniform(2.0, 20.0, events)
    frac = rng.uniform(0.0, 0.05, events)
    for i in range(events):
        P, S = shapes[kinds[i]]
        if dts[i] == 0:
            ev = _pulse_events(1, P, S, float(sig[i]), float(frac[i]), 250.0, g, device, 65535, torch.uint16)
        else:
            ev = _pulse_events(1, P, S, float(sig[i]), float(frac[i]), 250.0, g, device, (1 << 32) - 1,
                               torch.uint32)
        out.append(ev.reshape(P, S))
    return out


def laplace_blocks(n_blocks: int, L: int, dtype, seed: int = 5, device="cpu", outlier_rate: float = 1e-3,
                   const_rate: float = 0.01, full_rate: float = 0.01) -> torch.Tensor:
    """Stress data: per block round(centre + Laplace(0, s)), s ~ U(1, 50), centre at mid-range;
    outliers uniform over the whole dtype range at the given rate; a fraction of constant blocks
    (B = 1) and of full-range blocks (0 and 2^w - 1 forced)."""
    bits = {torch.uint8: 8, torch.uint16: 16, torch.uint32: 32}[dtype]
    maxv = (1 << bits) - 1
    g = _gen(seed, device)
    s = torch.rand(n_blocks, 1, generator=g, device=device, dtype=torch.float64) * 49.0 + 1.0
    u = torch.rand(n_blocks, L, generator=g, device=device, dtype=torch.float64) - 0.5
    lap = -s * torch.sign(u) * torch.log1p(-2.0 * u.abs())
    x = (float(1 << (bits - 1)) + lap).round_().clamp_(0, maxv)
    out_mask = torch.rand(n_blocks, L, generator=g, device=device) < outlier_rate
    outl = torch.floor(torch.rand(n_blocks, L, generator=g, device=device, dtype=torch.float64) * (maxv + 1.0))
    x = torch.where(out_mask, outl.clamp_(0, maxv), x)
    kind = torch.rand(n_blocks, generator=g, device=device)
    const = kind < const_rate
    full = (kind >= const_rate) & (kind < const_rate + full_rate)
    x[const] = x[const][:, :1].expand(-1, L) if int(const.sum()) else x[const]
    if int(full.sum()):
        xf = x[full]
        xf[:, 0] = 0
        xf[:, -1] = maxv
        x[full] = xf
    x = x.to(torch.int64)
    if dtype == torch.uint8:
        return x.to(torch.uint8)
    if dtype == torch.uint16:
        return x.to(torch.int32).to(torch.uint16)
    return x.to(torch.uint32)


def base_sweep_u32(L: int = 1024, lo: int = 2, hi: int = 1 << 16, seed: int = 7, device="cpu") -> torch.Tensor:
    """One u32 block per base B in [lo, hi]: values in [0, B-1] with 0 and B-1 both present."""
    g = _gen(seed, device)
    Bs = torch.arange(lo, hi + 1, device=device, dtype=torch.float64).reshape(-1, 1)
    x = torch.floor(torch.rand(Bs.shape[0], L, generator=g, device=device, dtype=torch.float64) * Bs)
    x[:, 0] = 0
    x[:, -1] = Bs[:, 0] - 1
    return x.to(torch.int64).to(torch.uint32).reshape(-1)


def paper_mixture(mu: float, sigma: float, x: float, y: float, a: int, N: int, rng: np.random.Generator):
    """Sec. 4.1 Eq. (12): N - a values from N(mu, sigma) and a values from U(x, y), at random
    positions, rounded and clipped at 0 (u32)."""
    v = np.empty(N, dtype=np.float64)
    v[: N - a] = rng.normal(mu, sigma, N - a)
    v[N - a:] = rng.uniform(x, y, a)
    rng.shuffle(v)
    return np.clip(np.round(v), 0, None).astype(np.uint32)


def nbytes_of(shapes_dtypes) -> int:
    return sum(math.prod(s) * d for s, d in shapes_dtypes)
