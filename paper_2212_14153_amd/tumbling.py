"""Tumbling analysis of fibers in shear flow (Sec. IV) from the fiber-ends recorder.

The recorder (Simulation.record / Batch.record, C ABI fpd_record_*) gives, every few steps,
each fiber's end-to-end vector e = R_last - R_first and centroid.  From it:

  theta(t)   the orientation of the fiber relative to +x (a director: theta and
             theta + pi are the same orientation), unwrapped continuously;
  omega(t)   d theta / dt; in the +-U channel the fiber turns clockwise (omega < 0);
  T          the tumbling period, the time to turn by pi (Sec. IV.B);
  L_ee       |e|, against the straight length (N - 1) l0 of the fiber;
  r_c fit    the aspect ratio that best fits omega(theta) to Jeffery's orbit, Eq. (19):
             omega = (gamma / 2) [(1 - r_c^2) / (1 + r_c^2) cos(2 theta) - 1],
             whose period is T = pi (r_c + 1 / r_c) / gamma.

The orbit is classified by the shape dynamics of Sec. IV.C (Fig. 7): a fiber that turns
little over the second half of the record is stuck (less than pi/8 and, given the shear
rate, a mean rate below 0.002 gamma over that half); a tumbling fiber whose end-to-end
length stays within 5 % of straight is on a Jeffery orbit, one that folds to between
60 % and 95 % makes S-turns, and one that folds further is S-coiled.  The paper
describes these orbits by their shapes and gives no numeric boundary, so the
thresholds are a reading.
"""
from __future__ import annotations

import math

import numpy as np

JEFFERY_MIN_LENGTH = 0.95   # min L_ee / straight length of a Jeffery orbit
S_TURN_MIN_LENGTH = 0.60    # ... of an S-turn; below it the fiber is S-coiled


def director_angle(ex, ey) -> np.ndarray:
    """Orientation in [-pi/2, pi/2] for the first sample, unwrapped with period pi (head and
    tail of the fiber are not told apart)."""
    a = np.arctan2(np.asarray(ey, dtype=float), np.asarray(ex, dtype=float))
    d = np.unwrap(2.0 * a) / 2.0
    return d - math.pi * round(d[0] / math.pi) if len(d) else d


def crossing_times(t, theta, step=math.pi):
    """Times at which theta passes theta[0] - k step (k = 1, 2, ...) going down, or
    theta[0] + k step going up, linearly interpolated."""
    t = np.asarray(t, dtype=float)
    theta = np.asarray(theta, dtype=float)
    sgn = -1.0 if theta[-1] < theta[0] else 1.0
    u = sgn * (theta - theta[0]) / step          # increasing overall
    out = []
    k = 1
    for i in range(1, len(u)):
        while u[i - 1] < k <= u[i]:
            f = (k - u[i - 1]) / (u[i] - u[i - 1])
            out.append(t[i - 1] + f * (t[i] - t[i - 1]))
            k += 1
    return np.array(out)


def jeffery_omega(theta, gamma: float, r_c: float):
    """Eq. (19)."""
    b = (1.0 - r_c * r_c) / (1.0 + r_c * r_c)
    return 0.5 * gamma * (b * np.cos(2.0 * np.asarray(theta)) - 1.0)


def jeffery_period(gamma: float, r_c: float) -> float:
    """Time to turn by pi on the orbit of Eq. (19)."""
    return math.pi * (r_c + 1.0 / r_c) / gamma


def fit_jeffery(theta, omega, gamma: float) -> float:
    """Least-squares r_c of Eq. (19) for samples omega(theta): omega is linear in
    B = (1 - r_c^2) / (1 + r_c^2), 2 omega / gamma + 1 = B cos(2 theta)."""
    c = np.cos(2.0 * np.asarray(theta))
    y = 2.0 * np.asarray(omega) / gamma + 1.0
    b = float(np.dot(c, y) / np.dot(c, c))
    b = min(max(b, -0.999999), 0.999999)
    return math.sqrt((1.0 - b) / (1.0 + b))


def analyse(record, fiber: int = 0, straight_length: float | None = None,
            gamma: float | None = None) -> dict:
    """Orbit quantities of one fiber from recorder rows [step, (ex, ey, cx, cy) ...]."""
    rec = np.asarray(record, dtype=float)
    t = rec[:, 0]
    ex, ey = rec[:, 1 + 4 * fiber], rec[:, 2 + 4 * fiber]
    theta = director_angle(ex, ey)
    omega = np.gradient(theta, t) if len(t) > 2 else np.zeros_like(t)
    lee = np.hypot(ex, ey)
    ref = straight_length if straight_length else float(lee[0])
    cross = crossing_times(t, theta)
    half = len(t) // 2
    out = {
        "t": t, "theta": theta, "omega": omega, "L_ee": lee,
        "turns": float(abs(theta[-1] - theta[0]) / math.pi),
        "period": float(np.mean(np.diff(cross))) if len(cross) >= 2 else float("nan"),
        "L_min": float(lee.min() / ref), "L_mean": float(lee.mean() / ref),
        "late_turn": float(abs(theta[-1] - theta[half])),
        "late_rate": float(abs(np.mean(omega[half:]))) if len(t) > 2 else 0.0,
    }
    if gamma:
        out["r_c_fit"] = fit_jeffery(theta, omega, gamma)
    return out


def final_angle_deg(a: dict) -> float:
    """The director's last orientation in degrees, in (-90, 90] (a stuck angle)."""
    th = math.degrees(float(a["theta"][-1]))
    return (th + 90.0) % 180.0 - 90.0


def turned_deg(a: dict) -> float:
    """Signed rotation over the record in degrees (negative: clockwise)."""
    return math.degrees(float(a["theta"][-1] - a["theta"][0]))


def classify(a: dict, gamma: float | None = None) -> str:
    """'stuck', 'jeffery', 's-turn' or 's-coiled' (see the module notes).  The record
    should span at least one expected tumbling period, else a slow turn looks stuck."""
    if a["late_turn"] < math.pi / 8 and (gamma is None or a["late_rate"] < 2e-3 * gamma):
        return "stuck"
    if a["L_min"] >= JEFFERY_MIN_LENGTH:
        return "jeffery"
    if a["L_min"] >= S_TURN_MIN_LENGTH:
        return "s-turn"
    return "s-coiled"
