"""Seeded synthetic processes: coupled AR pairs and 1/f (pink) noise ensembles.

Every generator returns float32 arrays shaped [R, T] (repetition-major), the
ensemble layout of the paper's Background section (observations x_t(r) of
repetition r at time t).  Recursions run in float64 and are rounded once to
float32 at the end.  Nothing here computes transfer entropy.
"""
from __future__ import annotations

import numpy as np

from .rng import derive_key, normal64

BURN_IN = 100   # samples simulated and discarded so every trial starts stationary


def _noise(key_ids, R: int, T: int) -> np.ndarray:
    return normal64(derive_key(*key_ids), R * T).reshape(R, T)


def coupled_ar(seed: int, R: int, T: int, *, a_x: float = 0.5, a_y: float = 0.5,
               coupling: float = 0.4, delay: int = 1, nonlinear: bool = False,
               burn_in: int = BURN_IN):
    """x_t = a_x x_{t-1} + e;  y_t = a_y y_{t-1} + c * f(x_{t-delay}) + e',  e, e' ~ N(0, 1).

    f is the identity (linear Gaussian pair) or tanh (nonlinear coupling).
    Returns (x, y) as float32 [R, T].
    """
    n = T + burn_in
    ex = _noise((seed, 1), R, n)
    ey = _noise((seed, 2), R, n)
    x = np.zeros((R, n))
    y = np.zeros((R, n))
    for t in range(n):
        xp = x[:, t - 1] if t >= 1 else 0.0
        yp = y[:, t - 1] if t >= 1 else 0.0
        x[:, t] = a_x * xp + ex[:, t]
        if t >= delay:
            drive = x[:, t - delay]
            if nonlinear:
                drive = np.tanh(drive)
        else:
            drive = 0.0
        y[:, t] = a_y * yp + coupling * drive + ey[:, t]
    return (x[:, burn_in:].astype(np.float32), y[:, burn_in:].astype(np.float32))


# Coupling scenarios of two AR(1) processes with time-varying coupling
# (Table 1; eq. 12-13 with the tanh profiles of eq. 14-16).  Time is in samples
# (1 kHz sampling, so one sample = 1 ms).
AR_SCENARIOS = {
    1: dict(alpha_x=0.75, alpha_y=0.35, beta_yx=0.0, beta_xy=-0.35, delta_yx=0, delta_xy=10),     # unidirectional
    2: dict(alpha_x=0.75, alpha_y=0.35, beta_yx=0.0, beta_xy=-0.35, delta_yx=0, delta_xy=10),     # two-step
    3: dict(alpha_x=0.475, alpha_y=0.35, beta_yx=-0.4, beta_xy=-0.35, delta_yx=20, delta_xy=10),  # bidirectional
}


def _tanh_step(t: np.ndarray, t0: float) -> np.ndarray:
    """0 -> 1 ramp with slope 0.05 per sample and inflection at t0 (eq. 14-15)."""
    return 0.5 * (1.0 + np.tanh(0.05 * (t - t0)))


def ar_scenario_couplings(scenario: int, t: np.ndarray):
    """gamma_XY(t), gamma_YX(t) of a scenario: eq. 15 (scenarios 1, 3), eq. 16 (scenario 2), eq. 14 (3)."""
    prm = AR_SCENARIOS[scenario]
    if scenario == 2:
        g_xy = prm["beta_xy"] * 0.5 * (_tanh_step(t, 1000.0) + _tanh_step(t, 2000.0))
    else:
        g_xy = prm["beta_xy"] * _tanh_step(t, 1000.0)
    g_yx = prm["beta_yx"] * _tanh_step(t, 2000.0)
    return g_xy, g_yx


def ar_scenario(seed: int, R: int, T: int, scenario: int, burn_in: int = BURN_IN):
    """x(t) = a_X x(t-1) + g_YX(t) y(t - d_YX) + n_X(t);  y(t) = a_Y y(t-1) + g_XY(t) x(t - d_XY) + n_Y(t)
    (eq. 12-13), unit-variance Gaussian noise, t = 0 .. T-1 after burn_in samples
    (the couplings are evaluated at negative times during the burn-in, where they vanish).
    Returns (x, y) as float32 [R, T].
    """
    prm = AR_SCENARIOS[scenario]
    n = T + burn_in
    t = np.arange(n, dtype=np.float64) - burn_in
    g_xy, g_yx = ar_scenario_couplings(scenario, t)
    ex = _noise((seed, 1), R, n)
    ey = _noise((seed, 2), R, n)
    x = np.zeros((R, n))
    y = np.zeros((R, n))
    dxy, dyx = prm["delta_xy"], prm["delta_yx"]
    for i in range(n):
        xp = x[:, i - 1] if i >= 1 else 0.0
        yp = y[:, i - 1] if i >= 1 else 0.0
        drive_x = g_yx[i] * y[:, i - dyx] if (prm["beta_yx"] != 0.0 and i >= dyx) else 0.0
        drive_y = g_xy[i] * x[:, i - dxy] if i >= dxy else 0.0
        x[:, i] = prm["alpha_x"] * xp + drive_x + ex[:, i]
        y[:, i] = prm["alpha_y"] * yp + drive_y + ey[:, i]
    return (x[:, burn_in:].astype(np.float32), y[:, burn_in:].astype(np.float32))


def pink_noise(seed_ids, R: int, T: int) -> np.ndarray:
    """Independent 1/f noise per repetition, float64 [R, T], zero mean, unit variance.

    White Gaussian noise is shaped in the frequency domain by amplitude f^(-1/2)
    (power 1/f) with the DC bin zeroed, then each repetition is standardised.
    """
    w = _noise(seed_ids, R, T)
    spec = np.fft.rfft(w, axis=1)
    f = np.fft.rfftfreq(T)
    gain = np.zeros_like(f)
    gain[1:] = f[1:] ** -0.5
    out = np.fft.irfft(spec * gain, n=T, axis=1)
    out -= out.mean(axis=1, keepdims=True)
    out /= out.std(axis=1, keepdims=True)
    return out


def switched_pink_pair(seed: int, R: int, T: int, *, coupling: float = 0.4, delay: int = 5,
                       on: int = 400, off: int = 800):
    """Pink source x and target y = n_y + c * x_{t-delay} for on <= t < off (0 elsewhere)."""
    x = pink_noise((seed, 11), R, T)
    ny = pink_noise((seed, 12), R, T)
    y = ny.copy()
    t = np.arange(T)
    gate = (t >= on) & (t < off) & (t >= delay)
    y[:, gate] += coupling * x[:, t[gate] - delay]
    return x.astype(np.float32), y.astype(np.float32)
