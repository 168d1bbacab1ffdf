"""Statistics of a cascade history used to compare runs that are not step
for step identical (test helper; pure numpy on history rows).

The quantities are those the paper reads off its runs:
  - growth rate of N- during the exponential phase (section 3, Eqs. 1-3),
  - the screening step, where <E> first changes sign (section 3),
  - the amplitude and frequency of the oscillation of <E> that follows
    (section 5, omega_0).
"""
import numpy as np


def growth_rate(n_minus, dt, n0):
    """Slope of ln N- against time over the exponential phase: the steps
    where N- lies between 20 N0 and a twentieth of its value at screening
    (least squares).  Returns (rate, first step, last step)."""
    n = np.asarray(n_minus, dtype=float)
    top = n.max()
    sel = np.nonzero((n >= 20.0 * n0) & (n <= top / 20.0))[0]
    if sel.size < 5:
        raise ValueError("no exponential phase")
    a, b = sel[0], sel[-1]
    t = np.arange(a, b + 1) * dt
    rate = np.polyfit(t, np.log(n[a:b + 1]), 1)[0]
    return float(rate), int(a), int(b)


def screening_step(e_mean):
    """First step at which <E> has changed sign from its start."""
    e = np.asarray(e_mean, dtype=float)
    s = np.sign(e[0]) if e[0] != 0 else 1.0
    idx = np.nonzero(np.sign(e) == -s)[0]
    if idx.size == 0:
        raise ValueError("no screening")
    return int(idx[0])


def oscillation(e_mean, dt, start, half_periods=8):
    """From step `start` (the screening step): the zero crossings of <E>
    (linear interpolation between steps), the angular frequency
    pi / mean half period over the first `half_periods` half periods, and the
    largest |<E>| over them.  Returns (omega, amplitude, crossings)."""
    e = np.asarray(e_mean, dtype=float)
    zs = []
    for k in range(max(start - 1, 0), len(e) - 1):
        if e[k] == 0.0 or (e[k] < 0) != (e[k + 1] < 0):
            frac = e[k] / (e[k] - e[k + 1]) if e[k] != e[k + 1] else 0.0
            zs.append(k + frac)
            if len(zs) > half_periods:
                break
    if len(zs) < half_periods + 1:
        raise ValueError("too few zero crossings")
    zs = np.array(zs)
    half = np.diff(zs).mean() * dt
    lo, hi = int(np.floor(zs[0])), int(np.ceil(zs[-1]))
    amp = float(np.abs(e[lo:hi + 1]).max())
    return float(np.pi / half), amp, zs
