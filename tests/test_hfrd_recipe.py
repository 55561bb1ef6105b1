"""The training-data perturbation of the paper's hybrid recipe (Sec. II.B,
Eqs. 3-6) and its constraint windows, on the CPU (no labels: those need DI)."""
import numpy as np
import pytest

from synth import mechanism as sm
from synth import workload as sw


@pytest.fixture(scope="module")
def base():
    m = sm.mech_medium()
    T0, p0, Y0, phi = sw.ignition_initial_states(m, 200, 11)
    # burnt-like states too, so that C and H sit in different species
    Tb, _, Yb, _ = sw.flame_block(m, 8, 12)
    return m, np.concatenate([T0, Tb]), np.full(T0.size + Tb.size, p0[0]), np.concatenate([Y0, Yb])


def test_element_ratios_of_fuel_air_and_air():
    m = sm.mech_medium()
    for phi in (0.5, 1.0, 1.5):
        Y = sw._mole_to_mass(sw.fuel_air_moles(m, np.array([phi])), m.W)
        hc, on, ph = sw.element_ratios(m, Y)[0]
        assert hc == pytest.approx(4.0, rel=1e-12)              # CH4
        assert on == pytest.approx(2.0 / (2 * 3.76), rel=1e-12)  # air
        assert ph == pytest.approx(phi, rel=1e-12)
    _, _, Ya = sw.air_states(m, 2)
    r = sw.element_ratios(m, Ya)
    assert np.isnan(r[0, 0]) and r[0, 2] == 0.0
    assert r[0, 1] == pytest.approx(2.0 / 7.52, rel=1e-12)


def test_zero_amplitudes_return_the_base_states(base):
    m, T, p, Y = base
    Tn, pn, Yn, b = sw.hfrd_states(m, T, p, Y, 500, 1, [None, None, None], alpha=0.0, beta=0.0,
                                   theta=0.0)
    assert np.array_equal(Tn, T[b]) and np.array_equal(pn, p[b])
    np.testing.assert_allclose(Yn, Y[b] / Y[b].sum(1, keepdims=True), rtol=0, atol=1e-16)


def test_perturbation_bounds_and_windows(base):
    m, T, p, Y = base
    win = [(2.65, 4.67), (0.254, 0.320), (0.2, 1.5)]
    Tn, pn, Yn, b = sw.hfrd_states(m, T, p, Y, 4000, 2, win)
    assert np.all(np.abs(Yn.sum(1) - 1.0) < 1e-14) and np.all(Yn >= 0.0)
    # Eq. 3: |T' - T| <= alpha (T_max - T_min); the draw fills the band
    d = np.abs(Tn - T[b]) / (T.max() - T.min())
    assert d.max() <= 0.125 + 1e-12 and d.max() > 0.12
    assert np.all((Tn >= 300.0) & (Tn <= 3000.0))
    # Eq. 4 at one pressure: the range is zero, so p' = p
    assert np.array_equal(pn, p[b])
    r = sw.element_ratios(m, Yn)
    for j, (lo, hi) in enumerate(win):
        assert np.all((r[:, j] >= lo) & (r[:, j] <= hi))


def test_species_exponent_and_n2_shift(base):
    """Eq. 6: Y'_j = Y_j^(1 + theta gamma) before normalisation, gamma in
    [-1, 1]; Eq. 5: Y'_N2 = Y_N2 + alpha gamma (range of Y_N2).  With alpha = 0
    the normalisation factor is Y_N2 / Y'_N2, which recovers the exponent."""
    m, T, p, Y = base
    n2 = sw._species_vec_index(m, N=2)
    Tn, pn, Yn, b = sw.hfrd_states(m, T, p, Y, 3000, 3, [None, None, None], alpha=0.0, beta=0.0)
    S = Y[b, n2] / Yn[:, n2]                      # unnormalised sum
    Yb = Y[b]
    mask = (Yb > 1e-30) & (Yb < 0.5)
    mask[:, n2] = False
    e = np.log(Yn[mask] * np.repeat(S[:, None], m.K, 1)[mask]) / np.log(Yb[mask])
    assert e.min() >= 0.9 - 1e-9 and e.max() <= 1.1 + 1e-9
    assert e.min() < 0.91 and e.max() > 1.09        # both ends of gamma reached
    # N2 alone, theta = 0: the unnormalised N2 moves by at most alpha times its range
    Tn, pn, Yn, b = sw.hfrd_states(m, T, p, Y, 3000, 4, [None, None, None], theta=0.0, beta=0.0)
    others = np.ones(m.K, bool)
    others[n2] = False
    S = Y[b][:, others].sum(1) / Yn[:, others].sum(1)     # the others are unchanged before normalising
    shift = (Yn[:, n2] * S - Y[b, n2]) / (Y[:, n2].max() - Y[:, n2].min())
    assert np.abs(shift).max() <= 0.125 + 1e-9 and np.abs(shift).max() > 0.12


def test_windows_that_exclude_everything_raise(base):
    m, T, p, Y = base
    with pytest.raises(RuntimeError):
        sw.hfrd_states(m, T, p, Y, 100, 5, [(10.0, 11.0), None, None], max_rounds=3)
