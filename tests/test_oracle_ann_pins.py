"""Pins of the oracle's learned-part reference (Box-Cox, GELU, MLP gradients,
Adam, bfloat16 rounding, element projection).  CPU only."""
import math

import numpy as np
import pytest

from oracle import ann
from synth import mechanism as sm


def test_box_cox_maps_unit_interval_as_stated():
    """Sec. II.B: mass fractions in [0, 1] map onto [-1/lambda, 0]."""
    assert ann.box_cox(0.0) == pytest.approx(-10.0, abs=0)
    assert ann.box_cox(1.0) == pytest.approx(0.0, abs=0)
    x = np.linspace(0, 1, 1001)
    f = ann.box_cox(x)
    assert np.all(np.diff(f) > 0) and f.min() >= -10.0 and f.max() <= 0.0
    # lambda -> 0 limit is the log branch of Eq. 7
    assert ann.box_cox(0.3, lam=1e-8) == pytest.approx(math.log(0.3), rel=1e-7)
    assert ann.box_cox(0.3, lam=0.0) == pytest.approx(math.log(0.3), rel=1e-15)
    assert ann.box_cox(-1e-12) == -10.0          # round-off negatives clamp to 0


def test_gelu_values():
    assert ann.gelu(0.0) == 0.0
    assert ann.gelu(1.0) == pytest.approx(0.8413447460685429, rel=1e-15)   # Phi(1)
    assert ann.gelu(-1.0) == pytest.approx(-0.15865525393145707, rel=1e-14)
    assert ann.gelu(10.0) == pytest.approx(10.0, rel=1e-15)
    assert abs(ann.gelu(-10.0)) < 1e-20
    x = np.linspace(-5, 5, 41)
    d = 1e-6
    fd = (ann.gelu(x + d) - ann.gelu(x - d)) / (2 * d)
    assert np.allclose(ann.gelu_grad(x), fd, rtol=1e-8, atol=1e-10)


def test_bf16_rounding_known_values():
    e = 2.0 ** -7                      # bfloat16 ulp at 1.0
    vals = np.array([1.0, 1 + e / 2, 1 + e / 2 + 2**-20, 1 + 3 * e / 2, -2.5, 3.0e38])
    want = np.array([1.0, 1.0, 1 + e, 1 + 2 * e, -2.5, 2.9942e38])
    got = ann.bf16(vals)
    assert got[0] == 1.0 and got[1] == 1.0          # tie to even
    assert got[2] == 1 + e and got[3] == 1 + 2 * e  # above the tie / tie to even (up)
    assert got[4] == -2.5
    assert got[5] == pytest.approx(want[5], rel=4e-3)


def test_mlp_backward_matches_finite_differences():
    dims = [6, 16, 12, 8, 3]
    Ws, bs = ann.init_params(dims, 1)
    rng = np.random.default_rng(2)
    bs = [rng.normal(0, 0.1, b.shape) for b in bs]
    X = rng.normal(size=(5, 6))
    tgt = rng.normal(size=(5, 3))
    out, cache = ann.forward(Ws, bs, X, quantize=False)
    loss, dout = ann.mse_loss(out, tgt)
    gW, gb = ann.backward(Ws, bs, cache, dout, quantize=False)

    def L(Ws_, bs_):
        o, _ = ann.forward(Ws_, bs_, X, quantize=False)
        return ann.mse_loss(o, tgt)[0]

    h = 1e-6
    for layer in range(len(Ws)):
        for (i, j) in [(0, 0), (1, 2), (Ws[layer].shape[0] - 1, Ws[layer].shape[1] - 1)]:
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[layer][i, j] += h
            Wm[layer][i, j] -= h
            fd = (L(Wp, bs) - L(Wm, bs)) / (2 * h)
            assert gW[layer][i, j] == pytest.approx(fd, rel=1e-6, abs=1e-10)
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[layer][1] += h
        bm[layer][1] -= h
        fd = (L(Ws, bp) - L(Ws, bm)) / (2 * h)
        assert gb[layer][1] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_adam_first_step_by_hand():
    """On f(x) = (x-3)^2 from x=0: g = -6, m1 = 0.1 g, v1 = 0.001 g^2; after
    bias correction the step is lr * g / (|g| + eps)."""
    lr = 0.01
    p, m, v = ann.adam_step(np.array([0.0]), np.array([-6.0]), np.zeros(1), np.zeros(1), 1, lr)
    assert m[0] == pytest.approx(-0.6, rel=1e-15)
    assert v[0] == pytest.approx(0.036, rel=1e-13)
    assert p[0] == pytest.approx(lr * 6.0 / (6.0 + 1e-8), rel=1e-13)


def test_projection_conserves_elements():
    mech = sm.mech_medium()
    E = ann.element_matrix(mech.composition, mech.element_mass)
    # every column of E sums to 1: a species' mass is carried by its elements
    assert np.allclose(E.sum(0), 1.0, rtol=1e-14)
    rng = np.random.default_rng(4)
    Y = rng.dirichlet(np.ones(mech.K), 8)
    dY = 1e-4 * rng.standard_normal(Y.shape)
    out = ann.project_delta(E, Y, dY)
    assert np.abs(out @ E.T).max() < 1e-18
    again = ann.project_delta(E, Y, out)
    assert np.abs(again - out).max() < 1e-19


def test_post_state_hand_computed_clipping():
    """One element carried by three species with equal weight (E = [1, 1, 1]),
    worked by hand.  y* = Y + dY = (0.6, 0.45, -0.02) has 0.03 too much mass;
    the first solve removes 0.01 from each species, leaving (0.59, 0.44, -0.03);
    the third is held at 0 and the second solve spreads the 0.05 excess of
    (0.6, 0.45, 0) over the other two: (0.575, 0.425, 0).  The whole
    correction is 0.025 / 0.1 = 0.25 of sd."""
    E = np.array([[1.0, 1.0, 1.0]])
    Y = np.array([[0.5, 0.5, 0.0]])
    dY = np.array([[0.1, -0.05, -0.02]])
    out, ok, adj = ann.post_state(E, Y, dY, np.full(3, 0.1))
    assert ok[0]
    assert np.allclose(out[0], [0.575, 0.425, 0.0], rtol=0, atol=1e-15)
    assert out[0, 2] == 0.0
    assert adj[0] == pytest.approx(0.25, rel=1e-13)
    # one solve only: the negative third species remains (and fails neg_tol)
    out1, ok1, _ = ann.post_state(E, Y, dY, np.full(3, 0.1), rounds=1)
    assert np.allclose(out1[0], [0.59, 0.44, -0.03], rtol=0, atol=1e-15) and not ok1[0]
    # unequal weights: the excess goes in proportion to sd^2
    out2, ok2, _ = ann.post_state(E, np.array([[0.5, 0.5, 0.0]]), np.array([[0.03, 0.0, 0.0]]),
                                  np.array([0.1, 0.2, 0.0 + 1e-12]))
    assert np.allclose(out2[0], [0.53 - 0.03 / 5, 0.5 - 0.03 * 4 / 5, 0.0], rtol=0, atol=1e-15)


def test_weighted_projection_solves_the_lagrange_system():
    """Without clipping, the correction is the minimiser of
    sum_k (y'_k - y*_k)^2 / sd_k^2 subject to E y' = E Y: checked against the
    stationarity (KKT) system [[diag(1/w), E^T], [E, 0]] [y'; lam] = [y*/w; E Y]
    solved as one dense linear system."""
    mech = sm.mech_medium()
    E = ann.element_matrix(mech.composition, mech.element_mass)
    rng = np.random.default_rng(8)
    Y = rng.dirichlet(np.ones(mech.K), 6)
    sd = 10.0 ** rng.uniform(-6, -2, mech.K)
    dY = 0.05 * sd * rng.standard_normal(Y.shape)
    out, ok, adj = ann.post_state(E, Y, dY, sd)
    assert ok.all()
    nE, K = E.shape
    for c in range(Y.shape[0]):
        w = sd * sd
        M = np.zeros((K + nE, K + nE))
        M[:K, :K] = np.diag(1.0 / w)
        M[:K, K:] = E.T
        M[K:, :K] = E
        rhs = np.concatenate([(Y[c] + dY[c]) / w, E @ Y[c]])
        sol = np.linalg.solve(M, rhs)
        assert np.allclose(out[c], sol[:K], rtol=1e-9, atol=1e-15)
        assert np.abs(E @ (out[c] - Y[c])).max() < 1e-15      # a few ulp of masses <= 1
        assert adj[c] == pytest.approx(np.max(np.abs(out[c] - Y[c] - dY[c]) / sd), rel=1e-12)


def test_post_state_holds_negatives_and_conserves():
    """Cold-cell-like states (six absent species) with noise: every result is
    non-negative, conserves the element masses to round-off, and leaves a
    species with a floored spread (inert in the training data) untouched."""
    mech = sm.mech_medium()
    E = ann.element_matrix(mech.composition, mech.element_mass)
    rng = np.random.default_rng(5)
    Y = rng.dirichlet(0.3 * np.ones(mech.K), 16)
    Y[:, :6] = 0.0
    Y /= Y.sum(1, keepdims=True)
    sd = 10.0 ** rng.uniform(-5, -3, mech.K)
    sd[10] = 1e-12
    dY = sd * rng.standard_normal(Y.shape)
    dY[:, 10] = 0.0
    out, ok, adj = ann.post_state(E, Y, dY, sd, neg_tol=0.0)
    assert (Y + dY < 0).any()
    assert ok.all() and out.min() >= 0.0
    m0 = Y @ E.T
    assert (np.abs((out - Y) @ E.T) / np.maximum(m0, 1e-300))[m0 > 1e-12].max() < 1e-13
    assert np.abs(out[:, 10] - Y[:, 10]).max() < 1e-20
    # against a general solver of the inequality-constrained problem (bounds
    # y' >= 0) where a single species was held: same minimiser
    from scipy.optimize import minimize
    for c in range(4):
        ys = Y[c] + dY[c]
        w = sd * sd
        r = minimize(lambda v: np.sum((v - ys) ** 2 / w) * 1e-6, np.maximum(out[c], 0),
                     jac=lambda v: 2e-6 * (v - ys) / w, method="SLSQP",
                     constraints=[{"type": "eq", "fun": lambda v: (E @ v - E @ Y[c]) * 1e3,
                                   "jac": lambda v: E * 1e3}],
                     bounds=[(0, None)] * mech.K, options={"ftol": 1e-20, "maxiter": 500})
        f_ours = np.sum((out[c] - ys) ** 2 / w)
        f_qp = np.sum((r.x - ys) ** 2 / w)
        assert f_ours <= f_qp * (1 + 1e-6) + 1e-12 or np.allclose(out[c], r.x, atol=1e-9)


# Standard normal CDF at 1 and 2.5, from printed tables of the normal
# distribution (independent of any erf routine): Phi(1), Phi(-2.5) = 1 - Phi(2.5).
PHI_1 = 0.8413447460685429
PHI_M2_5 = 0.0062096653257762


def _tiny_net():
    """A 2-2-1 network whose weights and input are exact in bfloat16."""
    W0 = np.array([[1.0, -1.0], [0.5, 2.0]])      # (in, out)
    b0 = np.array([0.25, -0.5])
    W1 = np.array([[2.0], [-1.0]])
    b1 = np.array([0.125])
    x = np.array([[1.0, -0.5]])
    return [W0, W1], [b0, b1], x


def test_forward_hand_computed_value():
    """Worked by hand: z0 = x W0 + b0 = (1 - 0.25 + 0.25, -1 - 1 - 0.5) = (1, -2.5);
    a0 = (1 Phi(1), -2.5 Phi(-2.5)); out = 2 a0[0] - a0[1] + 0.125."""
    Ws, bs, x = _tiny_net()
    out, cache = ann.forward(Ws, bs, x, quantize=False)
    assert np.array_equal(cache["Z"][0], [[1.0, -2.5]])
    a0 = np.array([PHI_1, -2.5 * PHI_M2_5])
    assert np.allclose(cache["A"][1], a0, rtol=1e-14, atol=0)
    want = 2.0 * a0[0] - a0[1] + 0.125
    assert out[0, 0] == pytest.approx(want, rel=1e-14)
    assert out[0, 0] == pytest.approx(1.823213655451526, rel=1e-14)


def test_forward_hand_computed_value_bf16():
    """The same network with the GPU's rounding points: the hidden activations
    are rounded to bfloat16 (8 significant bits).  a0[0] = 0.84134.. lies
    between 215/256 and 216/256 and rounds to 215/256 = 0.83984375;
    a0[1] = -0.0155241.. lies between 254 and 255 steps of 2^-14 and rounds
    to -254 * 2^-14 = -0.0155029296875.  Every other operand is exact, so
    out = 2 * 0.83984375 + 0.0155029296875 + 0.125 = 1.8201904296875 exactly."""
    Ws, bs, x = _tiny_net()
    out, cache = ann.forward(Ws, bs, x, quantize=True)
    assert np.array_equal(cache["A"][1], [[0.83984375, -0.0155029296875]])
    assert out[0, 0] == 1.8201904296875


# ---------------------------------------------------------------------------
# physics losses (Eqs. 9-11)
# ---------------------------------------------------------------------------
def test_phys_loss_without_weights_is_the_data_loss():
    rng = np.random.default_rng(1)
    o, t = rng.normal(size=(7, 5)), rng.normal(size=(7, 5))
    a, ga = ann.mse_loss(o, t)
    b, gb = ann.phys_loss(o, t, np.zeros(5), np.ones(5), None, 0.0, 0.0)
    assert a == b and np.array_equal(ga, gb)


def test_phys_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    B, K = 6, 4
    o, t = rng.normal(size=(B, K)), rng.normal(size=(B, K))
    mu, sd = rng.normal(0, 1e-3, K), rng.uniform(1e-3, 2e-3, K)
    G = rng.normal(size=(B, K))
    # keep every row's mass sum away from the kink of |m|
    o += (0.5 - (mu + sd * o).sum(1) / sd.sum())[:, None]
    f = lambda x: ann.phys_loss(x, t, mu, sd, G, 0.7, 0.3)[0]
    _, g = ann.phys_loss(o, t, mu, sd, G, 0.7, 0.3)
    h = 1e-6
    fd = np.zeros_like(o)
    for i in range(B):
        for k in range(K):
            e = np.zeros_like(o)
            e[i, k] = h
            fd[i, k] = (f(o + e) - f(o - e)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_output_weights_one_hot_uniform_and_by_hand():
    """Per-output weights of the data term: a one-hot w is the mean squared
    error of that column alone (the loss of a one-species network), uniform
    weights of any size give the plain mean, and a hand case."""
    rng = np.random.default_rng(3)
    B, K = 9, 6
    o, t = rng.normal(size=(B, K)), rng.normal(size=(B, K))
    for k in range(K):
        w = np.zeros(K)
        w[k] = 1.0
        loss, g = ann.phys_loss(o, t, np.zeros(K), np.ones(K), None, 0.0, 0.0, out_w=w)
        assert loss == pytest.approx(float(np.mean((o[:, k] - t[:, k]) ** 2)), rel=1e-14)
        assert np.all(g[:, np.arange(K) != k] == 0.0)
        np.testing.assert_allclose(g[:, k], 2.0 * (o[:, k] - t[:, k]) / B, rtol=1e-14)
    a, ga = ann.phys_loss(o, t, np.zeros(K), np.ones(K), None, 0.0, 0.0)
    b, gb = ann.phys_loss(o, t, np.zeros(K), np.ones(K), None, 0.0, 0.0, out_w=np.full(K, 3.5))
    assert b == pytest.approx(a, rel=1e-14)
    np.testing.assert_allclose(gb, ga, rtol=1e-14)
    # two rows, two outputs, w = (1, 3): d = ((1, 2), (0, -1)) ->
    # (1*1 + 3*4 + 0 + 3*1) / (2 * 4) = 16 / 8 = 2
    o2, t2 = np.array([[1.0, 2.0], [0.0, -1.0]]), np.zeros((2, 2))
    loss, g = ann.phys_loss(o2, t2, np.zeros(2), np.ones(2), None, 0.0, 0.0, out_w=[1.0, 3.0])
    assert loss == 2.0
    np.testing.assert_array_equal(g, [[2 * 1 * 1 / 8, 2 * 3 * 2 / 8], [0.0, 2 * 3 * -1 / 8]])


def test_species_networks_reproduce_the_k_output_network():
    """Splitting a K-output network into K one-output networks (hidden
    layers shared, output column k) must give the same outputs column by
    column: pins the column order of species_forward (a transposed stack, a
    shifted column or the wrong output slice fails)."""
    rng = np.random.default_rng(5)
    dims = [7, 12, 9, 5]
    Ws, bs = ann.init_params(dims, 3)
    bs = [rng.normal(0, 0.1, b.shape) for b in bs]
    X = rng.normal(size=(11, 7))
    for q in (False, True):
        full, _ = ann.forward(Ws, bs, X, quantize=q)
        sp = ann.species_forward(ann.species_split(Ws, bs), X, quantize=q)
        assert sp.shape == full.shape
        # equal up to the summation order of the library product
        np.testing.assert_allclose(sp, full, rtol=1e-13, atol=1e-15)
    # distinct networks: column k is network k's own forward, by hand for a
    # one-hidden-unit network with identity-like weights
    nets = []
    for k in range(3):
        W = [np.full((2, 1), float(k + 1)), np.array([[2.0]])]
        b = [np.zeros(1), np.array([float(k)])]
        nets.append((W, b))
    x = np.array([[1.0, 0.5]])
    out = ann.species_forward(nets, x, quantize=False)
    expect = [2.0 * ann.gelu(np.array(1.5 * (k + 1)))[()] + k for k in range(3)]
    np.testing.assert_allclose(out[0], expect, rtol=1e-15)


def test_weighted_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    B, K = 5, 4
    o, t = rng.normal(size=(B, K)), rng.normal(size=(B, K))
    w = rng.uniform(0.0, 2.0, K)
    f = lambda x: ann.phys_loss(x, t, np.zeros(K), np.ones(K), None, 0.0, 0.0, out_w=w)[0]
    _, g = ann.phys_loss(o, t, np.zeros(K), np.ones(K), None, 0.0, 0.0, out_w=w)
    h = 1e-6
    fd = np.zeros_like(o)
    for i in range(B):
        for k in range(K):
            e = np.zeros_like(o)
            e[i, k] = h
            fd[i, k] = (f(o + e) - f(o - e)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-10)


def test_mass_loss_by_hand_and_zero_when_mass_is_conserved():
    # two species, mu = (1e-3, -1e-3), sd = (1e-3, 2e-3): out = (1, 1) predicts
    # dY = (2e-3, 1e-3), sum 3e-3; |m| / sum(sd) = 3e-3 / 3e-3 = 1
    mu, sd = np.array([1e-3, -1e-3]), np.array([1e-3, 2e-3])
    o = np.array([[1.0, 1.0]])
    loss, _ = ann.phys_loss(o, o, mu, sd, None, 1.0, 0.0)
    assert loss == pytest.approx(1.0, rel=1e-12)
    # dY = (+d, -d) conserves mass: out = (d - mu) / sd per species
    d = 4e-3
    o2 = np.array([[(d - mu[0]) / sd[0], (-d - mu[1]) / sd[1]]])
    loss2, _ = ann.phys_loss(o2, o2, mu, sd, None, 1.0, 0.0)
    assert abs(loss2) < 1e-15


def test_heat_release_from_heats_of_formation():
    """At 298.15 K the species enthalpies are the heats of formation the
    tiny H/O mechanism was built from: moving mass from H2 + O2 to OH releases
    -sum_k h_f,k / W_k dY_k per unit mass."""
    from tests import mechs
    import oracle
    mech = mechs.tiny_hox()
    om = oracle.OracleMech(mech)
    hf = np.array([218e3, 249e3, 0.0, 0.0, 39e3])          # J/mol, as in tests/mechs.py
    W = om.W                                               # g/mol
    T, p, dt = np.array([298.15]), np.array([101325.0]), 1e-6
    Y = np.array([[0.0, 0.0, 0.2, 0.7, 0.1]])
    dY = np.array([[0.0, 0.0, -0.01, -0.02, 0.03]])
    G, s, hrr = ann.hrr_label_weights(om.species_thermo, W, T, p, Y, Y + dY, dt, np.ones(5))
    Wbar = 1.0 / (Y[0] / (W * 1e-3)).sum()
    rho = p[0] * Wbar / (8.31446261815324 * T[0])
    ref = -(rho / dt) * np.sum(hf / (W * 1e-3) * dY[0])
    assert hrr[0] == pytest.approx(ref, rel=1e-9)
    assert s == pytest.approx(abs(ref), rel=1e-12)


def test_heat_release_weights_identities():
    """With the frozen-chemistry prediction (dY* = 0) the normalised error is
    -HRR / s, and the labels' RMS is one in units of s."""
    from synth import mechanism as sm, workload as sw
    import oracle
    mech = sm.mech_medium()
    om = oracle.OracleMech(mech)
    T, p, Y = sw.uniform_cells(mech, 40, 8, T_range=(900, 2400))
    rng = np.random.default_rng(4)
    dY = rng.normal(0, 1e-4, Y.shape)
    dY -= dY.mean(1, keepdims=True)
    mu, sd = rng.normal(0, 1e-5, mech.K), rng.uniform(5e-5, 2e-4, mech.K)
    G, s, hrr = ann.hrr_label_weights(om.species_thermo, om.W, T, p, Y, Y + dY, 5e-7, sd)
    z = (dY - mu) / sd
    frozen = -mu / sd * np.ones_like(z)
    e = (G * (frozen - z)).sum(1)
    np.testing.assert_allclose(e, -hrr / s, rtol=1e-9, atol=1e-12)
    assert np.sqrt(np.mean((hrr / s) ** 2)) == pytest.approx(1.0, rel=1e-12)
