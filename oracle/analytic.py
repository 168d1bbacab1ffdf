"""Closed forms of arXiv:2012.05587 used to pin the oracle (test infrastructure).

Normalised units: c = m_e = e = omega_p0 = 1.  Gaussian 4*pi factors are
absorbed by omega_p0^2 = 4 pi e^2 n0 / m_e (section 3), so the screening
density of Eq. 5 reads n_s = E0^2 ln(2/f) / (2 gamma_thr) per species.
"""
import math

import numpy as np
from scipy.optimize import brentq
from scipy.special import lambertw


def t_accel(e0, gamma_thr):
    """t_a = gamma_thr m c / (e E0): time to reach threshold from rest (section 3)."""
    return gamma_thr / abs(e0)


def growth_rate_lambert(f, t_a):
    """Eq. 3 solved by the Lambert function: Gamma t_a = W(2/f) (small-f limit)."""
    return float(lambertw(2.0 / f).real) / t_a


def growth_rate_log(f, t_a):
    """The small-f approximation Gamma t_a ~ ln(2/f) stated after Eq. 3."""
    return math.log(2.0 / f) / t_a


def growth_rate_exact(f, t_a, tau=0.0):
    """Exponential root of the population model, Eqs. 1 and 2 of section 3.

    With n1, n2 ~ exp(Gamma t) and T = (1 - 3f/2) t_a, Eq. 1 gives
    n1 (e^{Gamma T} - 1) = (1 - f) n2 and Eq. 2 gives
    n2 (Gamma + 1/T) = 2 n1 / (f t_a), hence
        e^{Gamma T} - 1 = 2 (1 - f) / (f t_a (Gamma + 1/T)).
    tau > 0 is an extension for photons that convert after a mean delay tau
    (exponentially distributed): the pair source of Eq. 2 is then delayed,
    which multiplies it by 1 / (1 + Gamma tau) for exponential growth.  tau = 0
    is the paper's in-place model.
    """
    T = (1.0 - 1.5 * f) * t_a

    def h(G):
        return math.expm1(G * T) - 2.0 * (1.0 - f) / (f * t_a * (G + 1.0 / T) * (1.0 + G * tau))

    hi = 1.0 / T
    while h(hi) < 0.0:
        hi *= 2.0
    return brentq(h, 1e-12 / t_a, hi, xtol=1e-15, rtol=1e-14)


def screening_density(e0, gamma_thr, f):
    """Eq. 5, per species, normalised: n_s = E0^2 ln(2/f) / (2 gamma_thr)."""
    return e0 * e0 * math.log(2.0 / f) / (2.0 * gamma_thr)


def screening_time(e0, n0, growth):
    """t_s = (1/Gamma) ln(|E0| Gamma / (8 pi e c n0)) of section 3, normalised
    (8 pi e c n0 -> 2 n0 with n0 the seed density per species)."""
    return math.log(abs(e0) * growth / (2.0 * n0)) / growth


def mean_gamma(gamma_thr, f):
    """Eq. 10: <gamma> ~ gamma_thr / ln(2/f)."""
    return gamma_thr / math.log(2.0 / f)


def distribution_shape(gamma, gamma_thr, f):
    """Unnormalised Eq. 8: exp(-ln(2/f) gamma / gamma_thr)."""
    return np.exp(-math.log(2.0 / f) * np.asarray(gamma) / gamma_thr)


def relativistic_plasma_frequency(n_per_species, inv_gamma3):
    """Section 5: omega_0^2 = 8 pi e^2 n <1/gamma^3> / m, normalised 2 n <1/gamma^3>."""
    return math.sqrt(2.0 * n_per_species * inv_gamma3)


def leapfrog_cold_frequency(n_per_species, dt):
    """Discrete dispersion of the leapfrog-integrated cold pair plasma with a
    uniform field: sin(omega dt / 2) = omega_p dt / 2, omega_p^2 = 2 n."""
    wp = math.sqrt(2.0 * n_per_species)
    return 2.0 / dt * math.asin(wp * dt / 2.0)


def damped_field(t, e0p, eps0, omega0, inv_gamma3):
    """Eq. 24: <E>(t) under secondary bursts with constant eps0 (normalised)."""
    d = np.exp(-eps0 * omega0 * np.asarray(t) / (4.0 * math.pi))
    return e0p * d + 2.0 * omega0 / inv_gamma3 * (1.0 - d)
