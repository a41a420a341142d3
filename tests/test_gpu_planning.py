"""Trajectory planning with a learnable time interval (Sec. VII-A): controls
and (a, b) of Always_[aT, bT](inside Y) and Eventually(inside G) optimised
together, the STL term's gradients from the library.  The planted geometry is
synthetic (the paper does not give it), so the outcome is checked for the
properties the paper reports: the specification is met (robustness about 0
or above with the smooth operators), the interval grows beyond the nominal
size, the controls respect their limit.  Parity unpinned for the outcome; its
robustness and gradients are the library's, checked elsewhere against the
oracle."""
import numpy as np
import pytest
import torch

from paper_2501_04194_amd import planning

pytestmark = pytest.mark.gpu


def test_graph_step_matches_eager():
    _, a1, b1, r1, _ = planning.plan(steps=60, graph=False)
    _, a2, b2, r2, _ = planning.plan(steps=60, graph=True)
    assert np.allclose(a1, a2, atol=1e-4) and np.allclose(b1, b2, atol=1e-4) and np.allclose(r1, r2, atol=1e-3)


def test_planning_outcome():
    u, a, b, rho, dt = planning.plan(steps=2000, graph=True)
    assert (b - a > planning.I_NOM).all(), (a, b)
    assert (rho > -0.02).all(), rho
    assert float(torch.linalg.norm(u, dim=2).max()) <= planning.U_MAX + 0.05
    # the trajectory is inside Y over the chosen window and ends inside G
    x = planning.rollout(u, torch.zeros(u.shape[0], 2, device=u.device))[0].cpu().numpy()
    x0, x1, y0, y1 = planning.REGIONS["yellow"]
    lo, hi = int(np.ceil(a[0] * planning.T)) + 1, int(np.floor(b[0] * planning.T)) - 1
    seg = x[lo:hi + 1]
    assert ((seg[:, 0] > x0 - 0.05) & (seg[:, 0] < x1 + 0.05) & (np.abs(seg[:, 1]) < y1 + 0.05)).all()
