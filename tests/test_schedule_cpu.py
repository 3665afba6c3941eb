"""Host-side pieces of the learned schedule: protocol family, features, the ladder
efficiency and the Dinkelbach selection (checked against brute force over all
per-pair choices on a small grid, with a stand-in surrogate)."""
import itertools

import numpy as np

from paper_1006_4247_amd import schedule as sch


def test_protocol_endpoints_monotone_and_linear_limit():
    betas = np.array([1.0, 1.5, 2.5])
    K = np.array([3, 5])
    for g in (-2.0, 0.0, 2.0):
        lam = sch.protocol(betas, K, [g, g], 6)
        for i in range(2):
            pts = np.concatenate([[betas[i]], lam[i, : K[i]], [betas[i + 1]]])
            assert np.all(np.diff(pts) > 0)
    lin = sch.protocol(betas, K, [0.0, 0.0], 6)
    assert np.allclose(lin[0, :3], [1.125, 1.25, 1.375])
    assert np.all(lin[0, 3:] == 0)


def test_ladder_efficiency():
    assert abs(sch.ladder_efficiency([0.2, 0.4], [0, 0]) - 0.1) < 1e-15
    assert abs(sch.ladder_efficiency([1.0, 1.0, 1.0], [1, 2, 3]) - 0.15) < 1e-15


def test_dinkelbach_selection_is_optimal(monkeypatch):
    rng = np.random.default_rng(7)
    K_grid = [1, 2, 4, 8]
    gammas = (0.0, 1.0)
    R = 4
    table = {}

    def fake_predict(net, x):
        out = []
        for row in x:
            key = (round(float(row[0]), 6), int(round(row[5] * 32)), float(row[6]))
            if key not in table:
                k = key[1]
                table[key] = float(np.clip(rng.uniform(0.0, 0.6) * (1 - np.exp(-k / 3.0)), 0, 1))
            out.append(table[key])
        return np.array(out)

    monkeypatch.setattr(sch, "predict", fake_predict)
    betas = np.array([1.0, 1.3, 1.7, 2.2])
    ebar = np.array([-0.5, -0.6, -0.7, -0.8])
    K, G, A = sch.select_schedule(None, betas, ebar, 8, K_grid, gammas, floor=0.0)
    best = -1
    choices = [(k, g) for k in K_grid for g in gammas]
    for combo in itertools.product(choices, repeat=R - 1):
        acc = [fake_predict(None, sch.features(betas[i], betas[i + 1], ebar[i], ebar[i + 1], 8, k, g))[0]
               for i, (k, g) in enumerate(combo)]
        best = max(best, sch.ladder_efficiency(acc, [k for k, _ in combo]))
    got = sch.ladder_efficiency(A, K)
    assert abs(got - best) < 1e-12, (got, best)
