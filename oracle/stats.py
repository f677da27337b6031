"""Statistics derived from a neighbourhood function — TEST INFRASTRUCTURE ONLY.

Plain Python, loop by loop, following Section 4 ("Deriving useful data") and
Section 5 (spid) of the HyperANF paper:

* distance cdf H(t) = N(t) / max_t N(t);
* density h(t) = H(t) - H(t-1), with H(-1) = 0;
* effective diameter at alpha: the smallest t with H(t) >= alpha (alpha = 0.9 by default);
* interpolated effective diameter: the same crossing on the piecewise-linear
  interpolation of the points (t, H(t));
* average distance E = sum t h(t), variance sum t^2 h(t) - E^2, spid = variance / E;
* Algorithm 3: [D-, D+] with D- the largest t with N(t)/M <= alpha (1 - 2 eps) and D+
  the smallest t with N(t)/M >= alpha (1 + 2 eps).

Reading: N(t) counts pairs at distance <= t, self-pairs included (N(0) = n), and the
literal H above keeps them, so h(0) = n / max N. The ``distinct=True`` variant drops
them: H'(t) = (N(t) - N(0)) / (max N - N(0)).
"""
from __future__ import annotations

import math


def distance_cdf(nt, distinct: bool = False):
    nmax = max(nt)
    if distinct:
        base = nt[0]
        den = nmax - base
        if den <= 0:
            return [math.nan] * len(nt)
        return [(x - base) / den for x in nt]
    return [x / nmax for x in nt]


def density(H):
    out = []
    prev = 0.0
    for x in H:
        out.append(x - prev)
        prev = x
    return out


def effective_diameter(H, alpha: float = 0.9):
    for t, x in enumerate(H):
        if x >= alpha:
            return t
    return math.nan


def interpolated_effective_diameter(H, alpha: float = 0.9):
    t = effective_diameter(H, alpha)
    if isinstance(t, float) and math.isnan(t):
        return math.nan
    if t == 0:
        return 0.0
    return (t - 1) + (alpha - H[t - 1]) / (H[t] - H[t - 1])


def moments(h):
    mean = 0.0
    second = 0.0
    for t, x in enumerate(h):
        mean += t * x
        second += t * t * x
    return mean, second - mean * mean


def stats(nt, alpha: float = 0.9, distinct: bool = False):
    """Returns dict(ed, ied, avg_dist, var, spid, n_max, T)."""
    H = distance_cdf(nt, distinct)
    h = density(H)
    if distinct and len(h) and not math.isnan(H[0]):
        h[0] = 0.0  # no self-pairs in the distinct variant (undefined without any other pair)
    mean, var = moments(h)
    return dict(
        ed=effective_diameter(H, alpha),
        ied=interpolated_effective_diameter(H, alpha),
        avg_dist=mean,
        var=var,
        spid=(var / mean) if mean != 0 else math.nan,
        n_max=max(nt),
        T=len(nt) - 1,
    )


def diameter_interval(nt, eps: float, alpha: float = 0.9):
    """Algorithm 3: (D-, D+); None for a side that no t satisfies."""
    M = max(nt)
    lo = None
    hi = None
    for t, x in enumerate(nt):
        if x / M <= alpha * (1 - 2 * eps):
            lo = t
    for t, x in enumerate(nt):
        if x / M >= alpha * (1 + 2 * eps):
            hi = t
            break
    return lo, hi
