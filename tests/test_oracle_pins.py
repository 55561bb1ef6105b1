"""Pins of the FP64 oracle against facts fixed outside it: closed forms,
Rosenbrock order conditions, invariants, brute-force integration and textbook
special cases.  CPU only."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import oracle
from oracle import equilibrium as eq
from synth import mechanism as sm, workload as sw
from tests import mechs

RU = 8.31446261815324
RC = RU / 4.184
P = 101325.0


@pytest.fixture(scope="module")
def small():
    return oracle.OracleMech(sm.mech_small())


@pytest.fixture(scope="module")
def medium():
    return oracle.OracleMech(sm.mech_medium())


# ---------------------------------------------------------------- thermo ----
def test_nasa_constant_cp_closed_form():
    m = oracle.OracleMech(mechs.bimolecular())
    T = 1234.5
    cp, h, s = m.species_thermo(T)
    a6 = np.array([100.0, 300.0, 150.0, 250.0])
    a7 = np.array([2.0, 3.0, 4.0, 5.0])
    assert np.allclose(cp, 3.5, rtol=0, atol=1e-15)
    assert np.allclose(h, 3.5 + a6 / T, rtol=1e-15)
    assert np.allclose(s, 3.5 * math.log(T) + a7, rtol=1e-15)
    Y = np.array([0.1, 0.2, 0.3, 0.4])
    cpm, hm = m.cp_h(T, Y)
    Wkg = m.W * 1e-3
    assert cpm == pytest.approx(np.sum(Y * 3.5 * RU / Wkg), rel=1e-14)
    assert hm == pytest.approx(np.sum(Y * RU * (3.5 * T + a6) / Wkg), rel=1e-14)
    # T from h in closed form for constant cp
    h0 = hm
    T_exact = (h0 - np.sum(Y * RU * a6 / Wkg)) / np.sum(Y * 3.5 * RU / Wkg)
    Tn, rc = m.T_from_h(h0, Y, 500.0)
    assert rc == 0 and Tn == pytest.approx(T_exact, rel=1e-13)


def test_nasa_derivative_identities(medium):
    """dh/dT = cp and ds/dT = cp/T for every species (central differences)."""
    for T in (400.0, 1100.0, 2500.0):
        d = 1e-3
        cp, h, s = medium.species_thermo(T)
        _, hp, sp = medium.species_thermo(T + d)
        _, hm, smm = medium.species_thermo(T - d)
        dhdT = ((hp * (T + d)) - (hm * (T - d))) / (2 * d)     # d(h/R)/dT
        dsdT = (sp - smm) / (2 * d)
        assert np.allclose(dhdT, cp, rtol=1e-9)
        assert np.allclose(dsdT, cp / T, rtol=1e-8)


def test_cp_range_generator_contract(medium):
    for T in np.linspace(300, 3000, 28):
        cp, _, _ = medium.species_thermo(T)
        assert cp.min() >= 3.5 - 1e-9 and cp.max() <= 6.0 + 1e-9


def test_T_from_h_roundtrip(small):
    T, p, Y = sw.uniform_cells(small.src, 200, 7, T_range=(300, 3000))
    cp, h = small.thermo_batch(T, Y)
    T2, st = small.T_from_h_batch(h, Y, np.full(T.size, 1500.0))
    assert (st == 0).all()
    assert np.abs(T2 - T).max() < 1e-8


# ------------------------------------------------------------- integrator ----
def _rodas_std_form():
    g, A, C = oracle.rodas_coefficients()
    A6 = np.zeros((6, 6))
    C6 = np.zeros((6, 6))
    A6[:, :5] = A
    C6[:, :5] = C
    m = A6[5].copy()
    m[5] = 1.0
    mh = A6[4].copy()
    mh[4] = 1.0
    Gi = np.eye(6) / g - C6
    Gam = np.linalg.inv(Gi)
    alpha = A6 @ Gam
    return g, alpha, Gam, m @ Gam, mh @ Gam


def test_rodas_order_conditions():
    """Rosenbrock order conditions (Hairer & Wanner II, Table VI.7.1) up to order 4
    for the solution and order 3 for the embedded one."""
    g, alpha, Gam, b, bh = _rodas_std_form()
    beta = alpha + Gam - np.diag(np.diag(Gam))
    ai, bp = alpha.sum(1), beta.sum(1)

    def conds(w):
        return np.array([w.sum() - 1, w @ bp - (0.5 - g), w @ ai**2 - 1 / 3,
                         w @ (beta @ bp) - (1 / 6 - g + g * g), w @ ai**3 - 0.25,
                         w @ (ai * (alpha @ bp)) - (1 / 8 - g / 3),
                         w @ (beta @ ai**2) - (1 / 12 - g / 3),
                         w @ (beta @ (beta @ bp)) - (1 / 24 - g / 2 + 1.5 * g * g - g**3)])
    assert np.abs(conds(b)).max() < 1e-12
    assert np.abs(conds(bh)[:4]).max() < 1e-12
    assert np.abs(conds(bh)[4:]).max() > 1e-6      # the embedded method is only order 3


def test_rodas_empirical_order_linear():
    A = np.array([[-1.0, 0.5, 0.0], [-0.5, -1.0, 0.2], [0.1, 0.0, -2.0]])
    y0 = np.array([1.0, -0.5, 0.25])
    exact = expm(A) @ y0
    errs = []
    hs = [1 / 8, 1 / 16, 1 / 32, 1 / 64]
    for h in hs:
        y, rc, _ = oracle.rodas_generic(lambda y: A @ y, lambda y: A, y0, 1.0, 1e-10, 1e-10,
                                        fixed_h=h)
        assert rc == 0
        errs.append(np.abs(y - exact).max())
    slopes = np.diff(np.log(errs)) / np.diff(np.log(hs))
    assert slopes.min() > 3.7 and slopes.max() < 4.5


def test_rodas_stiff_decay_R_inf_zero():
    lam = 1e12
    y, rc, _ = oracle.rodas_generic(lambda y: -lam * y, lambda y: np.array([[-lam]]),
                                    np.array([1.0]), 1.0, 1e-10, 1e-10, fixed_h=1.0)
    assert rc == 0 and abs(y[0]) < 1e-9


def test_rodas_adaptive_nonlinear_exact():
    """y' = -y^2, y(0)=1 -> y = 1/(1+t)."""
    y, rc, cnt = oracle.rodas_generic(lambda y: -y * y, lambda y: np.array([[-2 * y[0]]]),
                                      np.array([1.0]), 3.0, 1e-14, 1e-11, h0=1e-3)
    assert rc == 0 and y[0] == pytest.approx(0.25, rel=1e-9)


# -------------------------------------------------------- closed forms --------
def _conc_M(T, p=P):
    return p / (RU * T) * 1e-6


def test_isomer_irreversible_closed_form():
    m = oracle.OracleMech(mechs.isomers(reversible=False))
    T0, dt = 1500.0, 1e-6
    kf = math.exp(math.log(1e13) - 5000.0 / (RC * T0))
    Y0 = np.array([[0.9, 0.1]])
    T, Y, st, _ = m.advance(np.array([T0]), P, Y0, dt, rtol=1e-12, atol_Y=1e-20)
    ya = 0.9 * math.exp(-kf * _conc_M(T0) * dt)
    assert st[0] == 0
    assert Y[0, 0] == pytest.approx(ya, rel=1e-9)
    assert Y[0, 1] == pytest.approx(1.0 - ya, rel=1e-9)
    assert T[0] == pytest.approx(T0, rel=1e-13)


def test_isomer_reversible_closed_form():
    gap = 0.7                                   # s_B - s_A in units of R
    m = oracle.OracleMech(mechs.isomers(reversible=True, s_gap=gap))
    T0, dt = 1300.0, 2e-6
    kf = math.exp(math.log(1e13) - 5000.0 / (RC * T0))
    Kc = math.exp(gap)
    kr = kf / Kc
    y_eq = 1.0 / (1.0 + Kc)
    T, Y, st, _ = m.advance(np.array([T0]), P, np.array([[0.95, 0.05]]), dt, rtol=1e-12,
                            atol_Y=1e-20)
    ya = y_eq + (0.95 - y_eq) * math.exp(-(kf + kr) * _conc_M(T0) * dt)
    assert st[0] == 0
    assert Y[0, 0] == pytest.approx(ya, rel=1e-9)


def test_bimolecular_closed_form():
    """A + B -> C + D at constant T and rho (zero reaction enthalpy, dnu = 0):
    C_A(t) = C_A0 (C_B0 - C_A0) / (C_B0 exp((C_B0 - C_A0) k t) - C_A0)."""
    m = oracle.OracleMech(mechs.bimolecular())
    T0, dt = 1400.0, 5e-6
    k = math.exp(math.log(3e12) + 0.5 * math.log(T0) - 4000.0 / (RC * T0))
    Y0 = np.array([0.05, 0.6, 0.15, 0.2])
    W = m.W
    Wbar = 1.0 / np.sum(Y0 / W)
    rho = P * Wbar * 1e-3 / (RU * T0)                        # kg/m^3
    C0 = rho * Y0 / (W * 1e-3) * 1e-6                        # mol/cm^3
    a, b = C0[0], C0[1]
    ca = a * (b - a) / (b * math.exp((b - a) * k * dt) - a)
    T, Y, st, _ = m.advance(np.array([T0]), P, Y0[None], dt, rtol=1e-12, atol_Y=1e-20)
    ya = ca * 1e6 * W[0] * 1e-3 / rho
    assert st[0] == 0
    assert Y[0, 0] == pytest.approx(ya, rel=1e-9)
    assert T[0] == pytest.approx(T0, rel=1e-12)


# ------------------------------------------------------------ jacobian -------
@pytest.mark.parametrize("which", ["small", "medium"])
def test_jacobian_matches_finite_differences(which, small, medium):
    m = small if which == "small" else medium
    T, p, Y = sw.uniform_cells(m.src, 3, 11, T_range=(1000, 2200))
    for c in range(3):
        y = np.r_[Y[c], T[c]]
        J = m.jacobian(y, p[c])
        N = y.size
        Jfd = np.zeros((N, N))
        for j in range(N):
            hstep = 1e-5 * max(abs(y[j]), 1e-6) if j < N - 1 else 1e-3
            cols = []
            for hh in (hstep, hstep / 2):
                yp, ym = y.copy(), y.copy()
                yp[j] += hh
                ym[j] -= hh
                cols.append((m.rhs(yp, p[c]) - m.rhs(ym, p[c])) / (2 * hh))
            Jfd[:, j] = (4 * cols[1] - cols[0]) / 3        # Richardson
        scale = np.abs(Jfd).max(axis=1, keepdims=True)
        err = np.abs(J - Jfd) / (np.abs(Jfd) + 1e-6 * scale + 1e-300)
        assert err.max() < 1e-5


# ------------------------------------------------------------ equilibrium ----
def test_gibbs_isomers_closed_form():
    gap = 0.9
    m = oracle.OracleMech(mechs.isomers(reversible=True, s_gap=gap))
    n = eq.equilibrium_TP(m, 1500.0, P, np.array([2.0]))
    assert n[1] / n[0] == pytest.approx(math.exp(gap), rel=1e-10)
    assert n.sum() == pytest.approx(1.0, rel=1e-12)


def test_gibbs_dissociation_quadratic():
    """H2 = 2H: x_H^2/x_H2 = K_p (p0/p) -> quadratic for x_H."""
    mech = mechs.tiny_hox()
    m = oracle.OracleMech(mech)
    T = 3200.0
    b = np.array([2.0, 1e-300])
    n = eq.equilibrium_TP(m, T, P, b)
    _, hRT, sR = m.species_thermo(T)
    g = hRT - sR
    Kp = math.exp(-(2 * g[0] - g[2]))
    # x_H^2 = Kp (1 - x_H) at p = p0
    xH = (-Kp + math.sqrt(Kp * Kp + 4 * Kp)) / 2
    x = n / n.sum()
    assert x[0] == pytest.approx(xH, rel=1e-9)


def test_detailed_balance_at_gibbs_equilibrium(small):
    T = 2100.0
    _, _, Y = sw.uniform_cells(small.src, 1, 5)
    b = eq.element_moles(small, Y[0])
    n = eq.equilibrium_TP(small, T, P, b, x0=np.full(small.K, 1.0 / small.K))
    Ye = n * small.W
    Ye /= Ye.sum()
    qf, qr = small.fluxes(T, P, Ye)
    rel = np.abs(qf - qr) / np.maximum(qf, 1e-300)
    assert rel.max() < 1e-9


# ---------------------------------------------------------------- invariants --
def test_conservation_and_enthalpy_closure(small):
    """Without projection: element masses drift only by round-off, and the
    integrated T agrees with the T recovered from the conserved enthalpy
    (this pins the sign and scale of the energy equation)."""
    T, p, Y = sw.uniform_cells(small.src, 16, 2001)
    T1, Y1, st, _ = small.advance(T, p, Y, 1e-6, rtol=1e-10, project=False, newton_T=False)
    assert (st == 0).all()
    for c in range(16):
        m0, m1 = small.element_mass(Y[c]), small.element_mass(Y1[c])
        assert np.all(np.abs(m1 - m0) <= 1e-12 * m0 + 1e-18)
        cp0, h0 = small.cp_h(T[c], Y[c])
        Tn, rc = small.T_from_h(h0, Y1[c], T1[c])
        assert rc == 0 and abs(Tn - T1[c]) < 10 * 1e-10 * T1[c] + 1e-6
    assert np.abs(Y1.sum(1) - 1).max() < 1e-13


def test_tolerance_self_consistency(small):
    T, p, Y = sw.uniform_cells(small.src, 8, 2001)
    Ta, Ya, _, _ = small.advance(T, p, Y, 1e-6, rtol=1e-10)
    Tb, Yb, _, _ = small.advance(T, p, Y, 1e-6, rtol=1e-12, atol_Y=1e-20, atol_T=1e-10)
    mask = Yb > 1e-8
    assert (np.abs(Ya - Yb)[mask] / Yb[mask]).max() < 1e-9
    assert np.abs(Ta - Tb).max() < 1e-6


def test_relaxation_to_gibbs_equilibrium():
    m = oracle.OracleMech(mechs.tiny_hox())
    T0 = np.array([2600.0])
    Y0 = np.array([[0.01, 0.02, 0.3, 0.6, 0.07]])
    T1, Y1, st, _ = m.advance(T0, P, Y0, 1.0, rtol=1e-11, atol_Y=1e-20)
    assert st[0] == 0
    cp, h0 = m.cp_h(T0[0], Y0[0])
    Te, Ye = eq.equilibrium_HP(m, h0, P, Y0[0], T_guess=T1[0])
    mask = Ye > 1e-8
    assert (np.abs(Y1[0] - Ye)[mask] / Ye[mask]).max() < 1e-6
    assert abs(T1[0] - Te) < 1e-3


def test_rk4_brute_force_tiny_mechanism():
    """Classical RK4 with dt/2^m until Richardson differences fall below 1e-12."""
    m = oracle.OracleMech(mechs.tiny_hox())
    y0 = np.array([0.002, 0.003, 0.1, 0.8, 0.095, 1800.0])
    y0[:5] /= y0[:5].sum()
    dt = 2e-6

    def rk4(nsteps):
        y = y0.copy()
        h = dt / nsteps
        for _ in range(nsteps):
            k1 = m.rhs(y, P)
            k2 = m.rhs(y + 0.5 * h * k1, P)
            k3 = m.rhs(y + 0.5 * h * k2, P)
            k4 = m.rhs(y + h * k3, P)
            y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        return y

    prev = rk4(256)
    for nst in (512, 1024, 2048, 4096):
        cur = rk4(nst)
        extrap = cur + (cur - prev) / 15.0
        if np.all(np.abs(cur - prev) / 15.0 <= 1e-12 * np.abs(cur)):
            break
        prev = cur
    T1, Y1, st, _ = m.advance(np.array([y0[5]]), P, y0[None, :5], dt, rtol=1e-12,
                              atol_Y=1e-22, atol_T=1e-10, project=False, newton_T=False)
    assert st[0] == 0
    assert np.allclose(Y1[0], extrap[:5], rtol=1e-9, atol=0)
    assert T1[0] == pytest.approx(extrap[5], rel=1e-11)


def test_projection_properties(small):
    _, _, Y = sw.uniform_cells(small.src, 4, 3)
    for c in range(4):
        ref = Y[c]
        pert = ref * (1 + 1e-6 * np.sin(np.arange(small.K) + c))
        out = small.project(ref, pert)
        assert np.abs(small.element_mass(out) - small.element_mass(ref)).max() < 5e-16
        out2 = small.project(ref, out)
        assert np.abs(out2 - out).max() < 5e-16            # P^2 = P
        same = small.project(ref, ref)
        assert np.abs(same - ref).max() < 5e-16            # conserving input unchanged
