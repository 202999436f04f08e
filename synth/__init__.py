"""Seeded synthetic inputs for MACH workloads.

This module is shared by the oracle-side tests and the GPU path.  It holds
input construction only (Gaussian draws, QR for random orthonormal factors,
the Tucker model of eq. tucker to build a test tensor, diurnal and spike
terms).  None of the method's arithmetic (coin toss, matricization,
HOSVD/HOOI) lives here.

Workloads (seed = 20260 + workload number unless overridden):
  1  dense FP64 64x32x48, Tucker core 5x5x5 N(0,1), random orthonormal
     factors, Gaussian noise sigma = 0.01 ||X_clean|| / sqrt(N); p = 0.1,
     rank (5,5,5), HOSVD + 10 sweeps.
  2  monitoring-shaped FP32 hosts x metrics x minutes 128x16x16384: Tucker
     rank (8,4,16) + per-host diurnal sinusoid (period 1440 minutes) + 0.1%
     Pareto(1.5) spikes; p in {0.1, 0.01}; rank (8,4,16); HOSVD + 20 sweeps.
  3  4-way FP32 64x64x64x256: core S x_n D with S ~ N(0,1) 10^4 and
     D = diag(0.8^0..0.8^9), relative noise 1e-2; p = 0.05, rank 10^4,
     HOSVD + 10 sweeps.
  4  workload 2's tensor with p in {0.2, 0.05, 0.01} x precision sweep.
  5  serving: Poisson arrivals (200/s) of hosts x 16 x T windows, hosts in
     {32, 64, 128}, T uniform in [1024, 16384], workload-1 style values at
     rank (8,4,16), p = 0.05, 8 streams.
The paper's own datasets (a 100x12x10080 machine-monitoring tensor and a
54x4x5385 sensor tensor, Section 4 Table 3) are not available; workloads 2
and 5 stand in for their shape (hosts x metrics x minute ticks, dense,
daily period).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "tucker_tensor", "workload1", "workload2",
    "workload3", "harmonic_tensor", "ServingRequest", "serving_stream",
    "serving_window", "scaled_shape",
]


@dataclass(frozen=True)
class Workload:
    name: str
    shape: tuple
    ranks: tuple
    ps: tuple
    sweeps: int
    dtype: str
    seed: int


WORKLOADS = {
    1: Workload("tucker-64x32x48-f64", (64, 32, 48), (5, 5, 5), (0.1,), 10, "f64", 20261),
    2: Workload("monitoring-128x16x16384-f32", (128, 16, 16384), (8, 4, 16), (0.1, 0.01), 20, "f32", 20262),
    3: Workload("voxel-64x64x64x256-f32", (64, 64, 64, 256), (10, 10, 10, 10), (0.05,), 10, "f32", 20263),
    4: Workload("monitoring-precision-sweep", (128, 16, 16384), (8, 4, 16), (0.2, 0.05, 0.01), 20, "f32", 20262),
}


def _orthonormal(rng, rows, cols):
    """Q factor of the QR of a rows x cols Gaussian matrix."""
    q, _ = np.linalg.qr(rng.standard_normal((rows, cols)))
    return q


def _tucker_product(core, factors):
    """core x_1 A1 x_2 A2 ... (the Tucker model, eq. tucker), built for input
    generation by successive tensordots."""
    X = np.asarray(core, dtype=np.float64)
    for n, A in enumerate(factors):
        X = np.moveaxis(np.tensordot(X, A, axes=([n], [1])), -1, n)
    return X


def tucker_tensor(shape, ranks, rng, core=None):
    """Noiseless Tucker tensor with random orthonormal factors.

    Returns (X, core, factors); factors[n] is I_n x R_n with orthonormal columns."""
    if core is None:
        core = rng.standard_normal(tuple(ranks))
    factors = [_orthonormal(rng, I, R) for I, R in zip(shape, ranks)]
    return _tucker_product(core, factors), core, factors


def workload1(shape=(64, 32, 48), ranks=(5, 5, 5), seed=20261, rel_noise=0.01,
              dtype=np.float64):
    """Tucker tensor + Gaussian noise, sigma = rel_noise * ||X_clean|| / sqrt(N)."""
    rng = np.random.default_rng(seed)
    Xc, core, factors = tucker_tensor(shape, ranks, rng)
    sigma = rel_noise * np.linalg.norm(Xc.ravel()) / np.sqrt(Xc.size)
    X = Xc + sigma * rng.standard_normal(shape)
    return X.astype(dtype), factors


def workload2(shape=(128, 16, 16384), ranks=(8, 4, 16), seed=20262, period=1440.0,
              spike_frac=1e-3, pareto_alpha=1.5):
    """Monitoring-shaped hosts x metrics x minutes tensor, float32.

    Tucker part: N(0,1) core, random orthonormal factors.
    Diurnal part: a_h sin(2 pi t / period + phi_h) m_j with a_h ~ U[0.5, 1.5]
    times the Tucker RMS, phi_h ~ U[0, 2 pi), m a fixed unit metric profile.
    Spikes: a fraction spike_frac of entries (chosen by an independent
    generator) gets + x_m (1 + Lomax(alpha)) = classical Pareto(alpha, x_m),
    x_m = 3 x the Tucker RMS."""
    rng = np.random.default_rng(seed)
    Xc, _, factors = tucker_tensor(shape, ranks, rng)
    rms = np.linalg.norm(Xc.ravel()) / np.sqrt(Xc.size)
    H, M, T = shape
    a = rng.uniform(0.5, 1.5, H) * rms
    phi = rng.uniform(0.0, 2.0 * np.pi, H)
    m = rng.standard_normal(M)
    m /= np.linalg.norm(m)
    t = np.arange(T, dtype=np.float64)
    diurnal = np.sin(2.0 * np.pi * t[None, :] / period + phi[:, None]) * a[:, None]
    X = Xc + diurnal[:, None, :] * m[None, :, None]
    srng = np.random.default_rng(seed + 7919)
    n_spk = int(round(spike_frac * X.size))
    where = srng.choice(X.size, size=n_spk, replace=False)
    xm = 3.0 * rms
    X.ravel()[where] += xm * (1.0 + srng.pareto(pareto_alpha, n_spk))
    return X.astype(np.float32), factors


def workload3(shape=(64, 64, 64, 256), ranks=(10, 10, 10, 10), seed=20263,
              ratio=0.8, rel_noise=1e-2):
    """4-way tensor with a geometrically decaying core spectrum, float32.

    core = S x_1 D x_2 D x_3 D x_4 D, S ~ N(0,1), D = diag(ratio^0..ratio^(R-1));
    noise sigma = rel_noise * ||X_clean|| / sqrt(N) (relative, as workload 1)."""
    rng = np.random.default_rng(seed)
    S = rng.standard_normal(tuple(ranks))
    core = S
    for n, R in enumerate(ranks):
        D = np.diag(ratio ** np.arange(R))
        core = np.moveaxis(np.tensordot(core, D, axes=([n], [1])), -1, n)
    Xc, _, factors = tucker_tensor(shape, ranks, rng, core=core)
    sigma = rel_noise * np.linalg.norm(Xc.ravel()) / np.sqrt(Xc.size)
    X = Xc
    X += sigma * rng.standard_normal(shape)
    return X.astype(np.float32), factors


def harmonic_tensor(n: int) -> np.ndarray:
    """x_ijk = 1 / (i + j + k), i, j, k = 1..n (Section 4, synthetic experiment)."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return 1.0 / (i[:, None, None] + i[None, :, None] + i[None, None, :])


def scaled_shape(shape, max_entries):
    """Shrink the largest modes (halving) until prod(shape) <= max_entries."""
    s = list(shape)
    while int(np.prod(s)) > max_entries:
        k = int(np.argmax(s))
        s[k] = max(1, s[k] // 2)
    return tuple(s)


# ---------------------------------------------------------------------------
# Workload 5: a Poisson stream of uneven windows
# ---------------------------------------------------------------------------


@dataclass(frozen=True)
class ServingRequest:
    req_id: int
    arrival_s: float
    stream_id: int
    window_id: int
    hosts: int
    T: int
    seed: int


def serving_stream(n_requests=1100, rate_per_s=200.0, n_streams=8, seed=20265,
                   hosts_choices=(32, 64, 128), t_lo=1024, t_hi=16384):
    """Seeded request list: exponential inter-arrival gaps (Poisson process),
    stream_id = request mod n_streams, hosts fixed per stream, T uniform."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, n_requests)
    arrivals = np.cumsum(gaps)
    hosts_of = rng.choice(hosts_choices, n_streams)
    Ts = rng.integers(t_lo, t_hi + 1, n_requests)
    win = [0] * n_streams
    out = []
    for r in range(n_requests):
        s = r % n_streams
        out.append(ServingRequest(r, float(arrivals[r]), s, win[s], int(hosts_of[s]),
                                  int(Ts[r]), seed * 1000 + s))
        win[s] += 1
    return out


def serving_window(req: ServingRequest, metrics=16, ranks=(8, 4, 16), rel_noise=0.01):
    """The hosts x metrics x T float32 window of a request.

    Host and metric factors and the core are fixed per stream (so a stream's
    windows share their host/metric subspaces); the time factor is new per
    window.  Noise sigma = rel_noise * ||X_clean|| / sqrt(N)."""
    srng = np.random.default_rng(req.seed)
    core = srng.standard_normal(tuple(ranks))
    A_h = _orthonormal(srng, req.hosts, ranks[0])
    A_m = _orthonormal(srng, metrics, ranks[1])
    wrng = np.random.default_rng([req.seed, req.window_id])
    A_t = _orthonormal(wrng, req.T, ranks[2])
    Xc = _tucker_product(core, [A_h, A_m, A_t])
    sigma = rel_noise * np.linalg.norm(Xc.ravel()) / np.sqrt(Xc.size)
    X = Xc + sigma * wrng.standard_normal(Xc.shape)
    return X.astype(np.float32)
