"""Seeded synthetic sparse-spectrum signals shaped like the paper's workload.

The paper's test signals (Sect. 5.1) place K frequencies uniformly at random
among the N, give each magnitude 1 and a uniform random phase, and leave the
other coefficients at zero (exactly sparse) or add white Gaussian noise at a
chosen SNR (general sparse).  This module draws such signals from a numpy
PCG64 generator and nothing else: it holds none of the sparse-FFT method's
arithmetic and is shared by the oracle side and the GPU side of every test.

Value convention: xhat = fft(x) / N, so a tone of amplitude a at frequency f
is x[n] = a * exp(+2 pi i f n / N).

Recipe (``Spec``):
  * positions: ``rng.choice(N, K, replace=False)``, sorted;
  * phases: U[0, 2 pi); magnitudes: 1 (``mag="unit"``) or 10**U[lo, hi]
    (``mag="loguniform"``);
  * SNR (dB) = 10 log10(mean |s|^2 / sigma^2) with mean |s|^2 = sum |a_f|^2,
    complex AWGN with E|n|^2 = sigma^2 (time domain);
  * x = N * ifft(xhat) (+ noise) in complex128, then cast to complex64.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Spec:
    N: int
    K: int
    seed: int
    mag: str = "unit"
    mag_lo: float = 0.0
    mag_hi: float = 2.0
    snr_db: float | None = None
    support: np.ndarray = field(default=None, repr=False)
    values: np.ndarray = field(default=None, repr=False)

    @property
    def noise_var(self) -> float:
        if self.snr_db is None:
            return 0.0
        p = float(np.sum(np.abs(self.values) ** 2))
        return p / (10.0 ** (self.snr_db / 10.0))


def make_spec(N: int, K: int, seed: int, mag: str = "unit", mag_lo: float = 0.0,
              mag_hi: float = 2.0, snr_db: float | None = None, support=None,
              values=None) -> Spec:
    """Draw the sparse spectrum (positions and values) of one signal."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if support is None:
        support = np.sort(rng.choice(N, size=K, replace=False)).astype(np.int64)
    else:
        support = np.asarray(support, dtype=np.int64)
    if values is None:
        phase = rng.uniform(0.0, 2.0 * np.pi, size=len(support))
        if mag == "unit":
            amp = np.ones(len(support))
        elif mag == "loguniform":
            amp = 10.0 ** rng.uniform(mag_lo, mag_hi, size=len(support))
        else:
            raise ValueError(mag)
        values = amp * np.exp(1j * phase)
    return Spec(N=N, K=K, seed=seed, mag=mag, mag_lo=mag_lo, mag_hi=mag_hi,
                snr_db=snr_db, support=support, values=np.asarray(values, np.complex128))


def synth(spec: Spec) -> np.ndarray:
    """complex64 time signal of ``spec`` on the host (numpy)."""
    N = spec.N
    xh = np.zeros(N, dtype=np.complex128)
    xh[spec.support] = spec.values
    x = np.fft.ifft(xh) * N
    if spec.snr_db is not None:
        rng = np.random.Generator(np.random.PCG64(spec.seed ^ 0x5EED5EED))
        s = np.sqrt(spec.noise_var / 2.0)
        x = x + s * (rng.standard_normal(N) + 1j * rng.standard_normal(N))
    return x.astype(np.complex64)


def synth_torch(spec: Spec, device):
    """The same recipe evaluated with torch on ``device`` (used to fill large
    benchmark batches quickly).  The noise is drawn by torch's generator, so
    a noisy signal differs from :func:`synth`'s; every comparison that uses it
    hands the same array to both sides."""
    import torch
    N = spec.N
    xh = torch.zeros(N, dtype=torch.complex128, device=device)
    idx = torch.as_tensor(spec.support, device=device)
    xh[idx] = torch.as_tensor(spec.values, device=device)
    x = torch.fft.ifft(xh) * N
    if spec.snr_db is not None:
        g = torch.Generator(device=device)
        g.manual_seed(int(spec.seed) ^ 0x5EED5EED)
        s = float(np.sqrt(spec.noise_var / 2.0))
        nr = torch.randn(N, generator=g, device=device, dtype=torch.float64)
        ni = torch.randn(N, generator=g, device=device, dtype=torch.float64)
        x = x + s * torch.complex(nr, ni)
    return x.to(torch.complex64)


def truth(spec: Spec):
    """(support, values) of the planted spectrum, sorted by index."""
    o = np.argsort(spec.support)
    return spec.support[o], spec.values[o]
