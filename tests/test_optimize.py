"""Angle optimisation loop (host Adam on a batched value-and-gradient
callable), checked on the CPU against functions whose maxima are known: a
concave quadratic and the p=1 closed form on the 3-cube, whose optimum per
edge is 1/2 + 1/(3 sqrt 3) (tests/golden/qaoa_p1_known_values.json)."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import closed_form  # noqa: E402
import workloads  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CUBE = [(0, 1), (0, 2), (0, 4), (1, 3), (1, 5), (2, 3), (2, 6), (3, 7), (4, 5), (4, 6), (5, 7), (6, 7)]


def _opt():
    from paper_1709_03636_amd import optimize
    return optimize


def test_adam_on_concave_quadratic():
    a = torch.tensor([[0.3, -1.2], [2.0, 0.5], [-0.7, 0.0]], dtype=torch.float64)

    def vg(x):
        return -((x - a) ** 2).sum(1), -2.0 * (x - a)

    x0 = torch.zeros_like(a)
    xb, fb, trace = _opt().adam_maximize(vg, x0, steps=600, lr=0.05)
    assert torch.max(torch.abs(xb - a)) < 1e-3
    assert torch.all(fb <= 0) and torch.all(fb > -1e-6)
    assert trace.shape == (601,) and float(trace[-1]) >= float(trace[0])


def test_adam_reaches_p1_optimum_on_the_3cube():
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "qaoa_p1_known_values.json")))
    best = len(CUBE) * gold["triangle_free_3regular_max_edge_cost"]["value"]

    def vg(x):
        f, g = [], []
        for gam, bet in x.tolist():
            zz = closed_form.zz_p1(8, CUBE, gam, bet)
            dg, db = closed_form.zz_p1_grad(8, CUBE, gam, bet)
            f.append(float(np.sum((1 - zz) / 2)))
            g.append([-0.5 * dg.sum(), -0.5 * db.sum()])
        return torch.tensor(f, dtype=torch.float64), torch.tensor(g, dtype=torch.float64)

    x0 = torch.tensor(workloads.qaoa_angles(3, 6, 1), dtype=torch.float64)
    xb, fb, _ = _opt().adam_maximize(vg, x0, steps=400, lr=0.05)
    assert float(fb.max()) <= best + 1e-12
    assert float(fb.max()) >= best - 1e-6
    # the best point is a true maximiser of the closed form, not just a good value
    gam, bet = xb[int(fb.argmax())].tolist()
    assert abs(closed_form.cost_p1(8, CUBE, gam, bet) - float(fb.max())) < 1e-12
