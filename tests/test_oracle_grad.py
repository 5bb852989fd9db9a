"""Pins of the gradient oracle (CPU): the adjoint against the closed form of a single site
and against central differences of the plain current."""
import numpy as np
import pytest

pytest.importorskip("torch")

from oracle import dense as D  # noqa: E402
from oracle import grad as OG  # noqa: E402


def test_single_site_closed_form_gradient():
    # One site between wide-band leads (Gamma_L = Gamma_R = g_l): G = 1/(E - V + i G_t/2),
    # G_t = 2 g_l + gamma, T = (g_l G_t / 2) / ((E - V)^2 + G_t^2 / 4).
    gl, gam, V = 0.4, 0.3, 0.15
    E, w = D.midpoint_grid(-0.5, 0.5, 3)
    I, dV, dg = OG.adjoint(1, 1, 1.0, [V], [gam], E, w, lead_model=1, gamma_l=gl)
    Gt = 2 * gl + gam
    den = (E - V) ** 2 + Gt ** 2 / 4
    T = gl * Gt / 2 / den
    dT_dV = gl * Gt / 2 * 2 * (E - V) / den ** 2
    dT_dg = gl / 2 * (den - Gt ** 2 / 2) / den ** 2
    assert abs(I - np.dot(w, T)) < 1e-13
    assert abs(dV[0] - np.dot(w, dT_dV)) < 1e-12
    assert abs(dg[0] - np.dot(w, dT_dg)) < 1e-12


@pytest.mark.parametrize("h", [1e-5, 1e-6])
@pytest.mark.parametrize("W,L,lead_model,gamma_l", [(2, 3, 0, 0.0), (2, 3, 1, 0.7), (3, 1, 0, 0.0)])
def test_adjoint_matches_central_differences(W, L, lead_model, gamma_l, h):
    # h = 1e-6 is the step the differentiation workload names; 1e-5 checks that the agreement
    # does not hinge on one step size
    rng = np.random.default_rng(7)
    V = rng.uniform(-0.4, 0.4, W * L)
    g = rng.uniform(0.02, 0.3, W * L)
    E, w = D.midpoint_grid(-1.7, 1.3, 3)
    I, dV, dg = OG.adjoint(W, L, 1.0, V, g, E, w, lead_model, 1e-10, gamma_l)
    sols = D.solve_workload(W, L, 1.0, V, g, E, lead_model, 1e-10, gamma_l)
    assert abs(I - D.current(sols, w)) < 1e-12 * abs(I)
    fV = OG.central_differences(W, L, 1.0, V, g, E, w, h, lead_model, 1e-10, gamma_l, "V")
    fg = OG.central_differences(W, L, 1.0, V, g, E, w, h, lead_model, 1e-10, gamma_l, "gamma")
    scale = max(np.abs(dV).max(), np.abs(dg).max())
    assert np.abs(dV - fV).max() < 1e-7 * scale
    assert np.abs(dg - fg).max() < 1e-7 * scale
