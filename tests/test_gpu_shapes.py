"""The tumbling and stuck fibers of Sec. IV on the GPU path, against what the paper
prints: the stuck angles of Fig. 7 and the sense and amount of rotation of Fig. 9
(tests/golden/stuck_fibers.txt), and the critical Re_ps and C of Figs. 5 and 8 with the
scaling of the rigid fiber's period below Re_cr (tests/golden/critical_values.txt); each
row of the fixtures names its figure.

These are loose checks of the physics (the paper's values come from one resolution and
are read from captions), not parity: no oracle run of 400k steps on these lattices
finishes in test time.  Angles are held to 1.5 degrees, rotations to 15 degrees, the
period ratio to 10 %.  All runs share one batch, FP32 storage, recorded every 200 steps.
"""
import math
import os

import numpy as np
import pytest

import workloads
from paper_2212_14153_amd import _lib, tumbling

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(__file__), "golden")
GAMMA = 1.5e-4
STEPS = 400000
EVERY = 200


def table(name):
    rows = []
    for line in open(os.path.join(HERE, name)):
        if line.strip() and not line.startswith("#"):
            rows.append(line.split())
    return rows


def stuck_rows():
    return [dict(K=float(k), Re=float(re), C=float(c), theta=float(th), sense=sense,
                 turned=None if turned == "-" else float(turned))
            for k, re, c, th, sense, turned, *_ in table("stuck_fibers.txt")]


def critical_rows():
    return [dict(q=q, K=float(k), other=float(o), value=float(v), below=float(lo),
                 above=float(hi)) for q, k, o, v, lo, hi, *_ in table("critical_values.txt")]


def key_of(row, x):
    """(K, Re_ps, C) of a bracketing run."""
    return (row["K"], x, row["other"]) if row["q"] == "Re_cr" else (row["K"], row["other"], x)


@pytest.fixture(scope="module")
def runs():
    """(K, Re_ps, C) -> analysis of its record."""
    keys = [(r["K"], r["Re"], r["C"]) for r in stuck_rows()]
    for r in critical_rows():
        keys += [key_of(r, r["below"]), key_of(r, r["above"])]
    keys.append((33.0, 1.0, 0.2))        # for the period ratio below Re_cr
    keys = list(dict.fromkeys(keys))
    ws = [workloads.flexible_fiber(k, c, re, gamma=GAMMA, steps=STEPS) for k, re, c in keys]
    params = [_lib.params_from_mapping(w.params(), storage="f32") for w in ws]
    print(f"[case] tumbling and stuck fibers: {len(ws)} runs, {STEPS} steps", flush=True)
    budget = int(1.1 * sum(_lib.fpd_sim_footprint(p) for p in params)) + (1 << 26)
    out = {}
    with _lib.Batch(budget, len(ws), storage="f32") as b:
        ids = [b.add(p, w.beads(), STEPS) for p, w in zip(params, ws)]
        for sid in ids:
            b.record_start(sid, EVERY, STEPS // EVERY + 8)
        while b.run(50000):
            pass
        for key, w, sid in zip(keys, ws, ids):
            assert b.info(sid)[1] == _lib.FPD_SIM_DONE, key
            out[key] = tumbling.analyse(b.record(sid), gamma=GAMMA,
                                        straight_length=(w.n_beads - 1) * w.l0)
    return out


@pytest.mark.parametrize("row", stuck_rows(),
                         ids=lambda r: f"K{r['K']:g}_Re{r['Re']:g}_C{r['C']:g}")
def test_stuck_angle_and_rotation(runs, row):
    a = runs[(row["K"], row["Re"], row["C"])]
    assert tumbling.classify(a, GAMMA) == "stuck"
    assert abs(tumbling.final_angle_deg(a) - row["theta"]) <= 1.5
    turned = tumbling.turned_deg(a)
    assert (turned < 0) == (row["sense"] == "cw")
    if row["turned"] is not None:
        assert abs(abs(turned) - row["turned"]) <= 15.0


@pytest.mark.parametrize("row", critical_rows(),
                         ids=lambda r: f"{r['q']}_K{r['K']:g}_{r['value']:g}")
def test_critical_value_is_bracketed(runs, row):
    assert row["below"] < row["value"] <= row["above"]
    below = runs[key_of(row, row["below"])]
    assert tumbling.classify(below, GAMMA) != "stuck"
    assert below["turns"] >= 0.9          # most of a half-turn or more
    assert tumbling.classify(runs[key_of(row, row["above"])], GAMMA) == "stuck"


def test_rigid_period_follows_the_square_root_law(runs):
    """gamma T ~ (Re_cr - Re_ps)^(-1/2) with the printed Re_cr = 2.2 (Fig. 5(b)): the first
    periods at Re_ps = 1 and 2 stand in the ratio ((2.2 - 1) / (2.2 - 2))^(1/2)."""
    def first_period(re):
        a = runs[(33.0, re, 0.2)]
        cross = tumbling.crossing_times(a["t"], a["theta"])
        assert len(cross) >= 1
        return cross[0]
    ratio = first_period(2.0) / first_period(1.0)
    assert ratio == pytest.approx(math.sqrt((2.2 - 1.0) / (2.2 - 2.0)), rel=0.10)
    assert np.isfinite(ratio)
