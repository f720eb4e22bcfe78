"""Source time functions (inputs only), sampled at t_k = k * dt for k = 1..n_steps.

The force applied in step k (the state at t_k) is wavelet[k - 1].
"""

from __future__ import annotations

import numpy as np


def ricker(n_steps: int, dt: float, f0: float, t0: float | None = None, amp: float = 1.0) -> np.ndarray:
    """Ricker wavelet (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2), tau = t - t0, t0 = 1.5 / f0."""
    if t0 is None:
        t0 = 1.5 / f0
    t = dt * np.arange(1, n_steps + 1, dtype=np.float64)
    a = (np.pi * f0 * (t - t0)) ** 2
    return amp * (1.0 - 2.0 * a) * np.exp(-a)


def sine_burst(n_steps: int, dt: float, f0: float, n_cycles: int = 2, amp: float = 1e12) -> np.ndarray:
    """amp * sin(w t) sin^2(w t / (2 n_c)) on [0, n_c / f0], zero afterwards (Section
    "Numerical implementation", the excitation signal)."""
    t = dt * np.arange(1, n_steps + 1, dtype=np.float64)
    w = 2 * np.pi * f0
    s = amp * np.sin(w * t) * np.sin(w * t / (2 * n_cycles)) ** 2
    s[t > n_cycles / f0] = 0.0
    return s
