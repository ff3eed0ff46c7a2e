"""Pins of the oracle's ROM trust-region driver (Algorithm 2, Sec. 4.3): the projection
onto the feasible set, the radius update, and the invariants the algorithm guarantees
(model exact at every centre, accepted steps decrease J, iterates feasible)."""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O
from oracle import tr as T
from oracle import filter as F
import workloads as W


def test_projection_matches_a_generic_qp_solver():
    rng = np.random.default_rng(0)
    for n, vmax in ((6, 2.0), (9, 4.5), (5, 10.0)):
        psi = rng.uniform(-0.5, 1.5, n)
        x = T.project_feasible(psi, vmax)
        res = minimize(lambda y: 0.5 * np.sum((y - psi) ** 2), np.full(n, min(0.5, vmax / n)),
                       jac=lambda y: y - psi, bounds=[(0, 1)] * n,
                       constraints=[{"type": "ineq", "fun": lambda y: vmax - y.sum(), "jac": lambda y: -np.ones(n)}],
                       method="SLSQP", options={"ftol": 1e-14, "maxiter": 500})
        assert np.abs(x - res.x).max() < 1e-6
        assert x.sum() <= vmax + 1e-12 and x.min() >= 0 and x.max() <= 1
    # KKT of the exact projection: x = clip(psi - lam), lam >= 0, volume active when lam > 0
    psi = rng.uniform(0, 1.2, 50)
    x = T.project_feasible(psi, 10.0)
    lam = np.median((psi - x)[(x > 0) & (x < 1)])
    assert lam >= 0 and np.allclose(x, np.clip(psi - lam, 0, 1), atol=1e-13)
    assert abs(x.sum() - 10.0) < 1e-12
    feas = np.full(8, 0.3)
    assert np.array_equal(T.project_feasible(feas, 5.0), feas)


def test_radius_update_follows_the_paper_constants():
    assert T.update_radius(2.0, -1.0, 100.0) == 1.0
    assert T.update_radius(2.0, 0.05, 100.0) == 1.0
    assert T.update_radius(2.0, 0.1, 100.0) == 2.0
    assert T.update_radius(2.0, 0.5, 100.0) == 2.0
    assert T.update_radius(2.0, 0.75, 100.0) == 4.0
    assert T.update_radius(80.0, 3.0, 100.0) == 100.0


@pytest.mark.parametrize("kind", ["res", "dist"])
def test_trust_region_invariants_on_mbb(kind):
    p = W.mbb2d(24, 8)
    prob = T.Problem(p.mesh, p.mask, p.f, F.filter_radius(1.5), 0.5)
    psi, hist = T.rom_tr(prob, kind=kind, tau=0.1, iters=4, window=4, nmax=3)
    assert psi.min() >= 0 and psi.max() <= 1 and psi.sum() <= prob.vmax + 1e-9
    J0 = hist[0]["J"]
    for h in hist:
        # Sec. 4.2: the basis holds the HDM state at the centre, so the model is exact there
        assert abs(h["model_center"] - h["J"]) <= 1e-9 * h["J"]
        if h["accepted"]:
            assert h["ratio"] >= T.ETA1 and h["J_cand"] < h["J"]
        assert h["model_cand"] <= h["model_center"]
    Jfinal = hist[-1]["J_cand"] if hist[-1]["accepted"] else hist[-1]["J"]
    assert Jfinal < J0
    assert any(h["accepted"] for h in hist)
    # the centre's J never increases
    centres = [h["J"] for h in hist]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(centres, centres[1:]))


def test_rejected_steps_keep_the_centre_and_halve_the_radius():
    """A one-column model (n_max = 0) and a large first radius: the first candidates
    increase J (ratio < 0), are rejected, and the radius halves until a step is accepted."""
    p = W.mbb2d(24, 8)
    prob = T.Problem(p.mesh, p.mask, p.f, F.filter_radius(1.5), 0.5)
    psi, hist = T.rom_tr(prob, kind="dist", tau=3.0, iters=4, window=2, nmax=0, move=0.5)
    assert [h["accepted"] for h in hist] == [False, False, False, True]
    for a, b in zip(hist, hist[1:]):
        if not a["accepted"]:
            assert b["J"] == a["J"] and b["delta"] == T.GAMMA1 * a["delta"]
    assert hist[0]["ratio"] < 0 and hist[-1]["J_cand"] < hist[0]["J"]
