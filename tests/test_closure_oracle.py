"""CPU pins of the oracle for the steps around the advance (oracle/closure.py):
transport mixing rules and the PaSR closure, and the synthetic transport
data they are fed."""
import numpy as np
import pytest

from oracle import closure as oc
from synth import mechanism as sm
from synth import transport as st
from synth import workload as sw


def test_chapman_enskog_nitrogen_at_room_temperature():
    """N2 with its tabulated Lennard-Jones parameters (3.621 A, 97.53 K):
    1.78e-5 Pa s is the measured viscosity at 300 K."""
    mu = st.viscosity_ce(28.014, 3.621, 97.53, np.array([300.0]))[0]
    assert mu == pytest.approx(1.78e-5, rel=0.02)


def test_ln_t_polynomials_reproduce_kinetic_theory():
    mech = sm.mech_medium()
    mu_c, lam_c = st.transport_fits(mech)
    W = mech.composition.astype(float) @ np.asarray(mech.element_mass, float)
    sig, eps = st.lennard_jones(mech)
    T = np.array([300.0, 700.0, 1500.0, 2900.0])
    mu = oc.poly_ln(mu_c, T)
    for k in range(mech.K):
        np.testing.assert_allclose(mu[:, k], st.viscosity_ce(W[k], sig[k], eps[k], T), rtol=0.01)
    assert np.all(oc.poly_ln(lam_c, T) > 0)


def test_mixing_rules_reduce_to_the_pure_species():
    rng = np.random.default_rng(1)
    K = 5
    W = rng.uniform(2.0, 44.0, K)
    mu = rng.uniform(1e-5, 8e-5, (1, K))
    lam = rng.uniform(0.02, 0.2, (1, K))
    for i in range(K):
        X = np.zeros((1, K))
        X[0, i] = 1.0
        assert oc.wilke(X, mu, W)[0] == pytest.approx(mu[0, i], rel=1e-14)
        assert oc.mathur_saxena(X, lam)[0] == pytest.approx(lam[0, i], rel=1e-14)
    # a species split in two identical halves is the same gas
    X2 = np.array([[0.3, 0.7]])
    assert oc.wilke(X2, np.array([[3e-5, 3e-5]]), np.array([28.0, 28.0]))[0] == pytest.approx(3e-5, rel=1e-14)
    # the conductivity average lies between the species values
    Xm = rng.dirichlet(np.ones(K), 10)
    lm = oc.mathur_saxena(Xm, np.repeat(lam, 10, 0))
    assert np.all(lm >= lam.min() - 1e-15) and np.all(lm <= lam.max() + 1e-15)


def _pasr_case(kscale=1.0):
    mech = sm.mech_medium()
    W = mech.composition.astype(float) @ np.asarray(mech.element_mass, float)
    T, p, Y0 = sw.uniform_cells(mech, 20, 5, T_range=(1200, 2200))
    rng = np.random.default_rng(6)
    dY = rng.normal(0, 1e-3, Y0.shape)
    dY -= dY.mean(1, keepdims=True)
    Y1 = np.clip(Y0 + dY, 0, None)
    Y1 /= Y1.sum(1, keepdims=True)
    k = np.full(20, 5.0) * kscale
    delta = np.full(20, 1e-3)
    mu = np.full(20, 6e-5)
    return mech, W, T, p, Y0, Y1, k, delta, mu


def test_pasr_limits_and_blend():
    mech, W, T, p, Y0, Y1, k, delta, mu = _pasr_case()
    dt = 1e-6
    kap, om, Yb = oc.pasr(W, T, p, Y0, Y1, dt, k, delta, mu)
    assert np.all((kap > 0) & (kap < 1))
    # the blend is a convex combination: sums to one
    np.testing.assert_allclose(Yb.sum(1), 1.0, rtol=0, atol=1e-13)
    # no turbulence: the reactor does not react; very intense mixing: kappa -> 1
    k0, _, Y0b = oc.pasr(W, T, p, Y0, Y1, dt, np.zeros(20), delta, mu)
    assert np.all(k0 == 0.0) and np.array_equal(Y0b, Y0)
    k_hi, _, _ = oc.pasr(W, T, p, Y0, Y1, dt, k * 1e12, delta, mu)
    assert np.all(k_hi > 0.99)
    # faster chemistry (same change over a shorter step: shorter tau_c) lowers kappa
    k_fast, _, _ = oc.pasr(W, T, p, Y0, Y1, dt / 10, k, delta, mu)
    assert np.all(k_fast < kap)
    # nothing forms: kappa = 1 and the source is the chemistry's
    k1, om1, _ = oc.pasr(W, T, p, Y0, Y0, dt, k, delta, mu)
    assert np.all(k1 == 1.0) and np.all(om1 == 0.0)
    # the source is kappa times rho dY/dt
    rho = oc.density(W, T, p, Y0)
    np.testing.assert_allclose(om, kap[:, None] * rho[:, None] * (Y1 - Y0) / dt, rtol=1e-15)
