"""GPU parity of the steps around the advance: transport properties and the
PaSR closure (csrc/closure.hip) against oracle/closure.py."""
import numpy as np
import pytest

from oracle import closure as oc
from synth import mechanism as sm
from synth import transport as st
from synth import workload as sw
from tests.gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("which", ["small", "medium", "large"])
def test_transport_matches_oracle(which):
    import torch
    from paper_2402_18858_amd import chemk
    mech = getattr(sm, f"mech_{which}")()
    ctx = chemk.Context(mech)
    mu_c, lam_c = st.transport_fits(mech)
    with pytest.raises(chemk.ChemkError) as e:
        ctx.transport(dev(np.array([1000.0])), dev(np.full((1, mech.K), 1.0 / mech.K)),
                      torch.zeros(1, dtype=torch.float64, device="cuda:0"))
    assert e.value.code == chemk.E_STATE
    ctx.transport_set(mu_c, lam_c)
    n = 1001   # ragged: not a multiple of the four cells per workgroup
    T, p, Y = sw.uniform_cells(mech, n, 31, T_range=(300, 3000))
    mu = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    lam = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    ctx.transport(dev(T), dev(Y), mu, lam)
    W = mech.composition.astype(float) @ np.asarray(mech.element_mass, float)
    mo, lo = oc.transport(mu_c, lam_c, W, T, Y)
    rm = np.abs(host(mu) / mo - 1).max()
    rl = np.abs(host(lam) / lo - 1).max()
    announce(f"transport {which}: {n} cells, max rel mu {rm:.2e}, lambda {rl:.2e}")
    assert rm < 1e-12 and rl < 1e-12


@pytest.mark.parametrize("which", ["medium", "large"])
def test_transport_at_block_size_matches_oracle_on_sampled_cells(which):
    """The full-block launch (several passes of each workgroup over its
    cells, and a ragged last pass) on 262,147 cells; the oracle on the first
    and last cells and a random sample between."""
    import torch
    from paper_2402_18858_amd import chemk
    mech = getattr(sm, f"mech_{which}")()
    ctx = chemk.Context(mech)
    mu_c, lam_c = st.transport_fits(mech)
    ctx.transport_set(mu_c, lam_c)
    n = 262_147
    T, p, Y = sw.uniform_cells(mech, n, 34, T_range=(300, 3000))
    mu = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    lam = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    ctx.transport(dev(T), dev(Y), mu, lam)
    rng = np.random.default_rng(35)
    idx = np.unique(np.concatenate([np.arange(40), np.arange(n - 40, n), rng.integers(0, n, 120)]))
    W = mech.composition.astype(float) @ np.asarray(mech.element_mass, float)
    mo, lo = oc.transport(mu_c, lam_c, W, T[idx], Y[idx])
    rm = np.abs(host(mu)[idx] / mo - 1).max()
    rl = np.abs(host(lam)[idx] / lo - 1).max()
    announce(f"transport {which}: {n} cells, {idx.size} sampled, max rel mu {rm:.2e}, lambda {rl:.2e}")
    assert rm < 1e-12 and rl < 1e-12


@pytest.mark.parametrize("which", ["small", "medium", "large"])
def test_pasr_matches_oracle(which):
    import torch
    from paper_2402_18858_amd import chemk
    mech = getattr(sm, f"mech_{which}")()
    ctx = chemk.Context(mech)
    W = mech.composition.astype(float) @ np.asarray(mech.element_mass, float)
    n = 777
    T, p, Y0 = sw.uniform_cells(mech, n, 32, T_range=(900, 2400))
    rng = np.random.default_rng(33)
    dY = rng.normal(0, 1e-3, Y0.shape)
    dY -= dY.mean(1, keepdims=True)
    Y1 = np.clip(Y0 + dY, 0, None)
    Y1 /= Y1.sum(1, keepdims=True)
    Y1[:5] = Y0[:5]                      # nothing forms: kappa = 1
    k = 10.0 ** rng.uniform(-1, 2, n)
    k[5:10] = 0.0                        # no sub-grid motion: kappa = 0
    delta = 10.0 ** rng.uniform(-4, -2.5, n)
    mu = rng.uniform(2e-5, 8e-5, n)
    dt = 1e-6
    kap = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    om = torch.zeros((n, mech.K), dtype=torch.float64, device="cuda:0")
    Yb = torch.zeros((n, mech.K), dtype=torch.float64, device="cuda:0")
    ctx.pasr(dev(T), dev(p), dev(Y0), dev(Y1), dt, dev(k), dev(delta), dev(mu), kappa=kap, omega=om, Y_out=Yb)
    ko, oo, yo = oc.pasr(W, T, p, Y0, Y1, dt, k, delta, mu)
    kg = host(kap)
    assert np.all(kg[:5] == 1.0) and np.all(kg[5:10] == 0.0)
    np.testing.assert_allclose(kg, ko, rtol=1e-12, atol=0)
    scale = np.abs(oo).max()
    np.testing.assert_allclose(host(om), oo, rtol=1e-11, atol=1e-13 * scale)
    np.testing.assert_allclose(host(Yb), yo, rtol=0, atol=1e-15)
    announce(f"PaSR: {n} cells, kappa in [{ko.min():.3f}, {ko.max():.3f}], max rel kappa "
             f"{np.abs(kg / np.where(ko > 0, ko, 1) - np.where(ko > 0, 1, 0)).max():.2e}")


@pytest.mark.parametrize("which", ["medium", "large"])
def test_pasr_at_block_size_matches_oracle_on_sampled_cells(which):
    """The full-block PaSR launch on 262,147 cells (a ragged last
    workgroup); the oracle on the first and last cells and a random sample."""
    import torch
    from paper_2402_18858_amd import chemk
    mech = getattr(sm, f"mech_{which}")()
    ctx = chemk.Context(mech)
    W = mech.composition.astype(float) @ np.asarray(mech.element_mass, float)
    n = 262_147
    T, p, Y0 = sw.uniform_cells(mech, n, 36, T_range=(900, 2400))
    rng = np.random.default_rng(37)
    dY = rng.normal(0, 1e-3, Y0.shape)
    dY -= dY.mean(1, keepdims=True)
    Y1 = np.clip(Y0 + dY, 0, None)
    Y1 /= Y1.sum(1, keepdims=True)
    k = 10.0 ** rng.uniform(-1, 2, n)
    delta = 10.0 ** rng.uniform(-4, -2.5, n)
    mu = rng.uniform(2e-5, 8e-5, n)
    dt = 1e-6
    kap = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    om = torch.zeros((n, mech.K), dtype=torch.float64, device="cuda:0")
    Yb = torch.zeros((n, mech.K), dtype=torch.float64, device="cuda:0")
    ctx.pasr(dev(T), dev(p), dev(Y0), dev(Y1), dt, dev(k), dev(delta), dev(mu), kappa=kap, omega=om, Y_out=Yb)
    idx = np.unique(np.concatenate([np.arange(40), np.arange(n - 40, n), rng.integers(0, n, 120)]))
    ko, oo, yo = oc.pasr(W, T[idx], p[idx], Y0[idx], Y1[idx], dt, k[idx], delta[idx], mu[idx])
    np.testing.assert_allclose(host(kap)[idx], ko, rtol=1e-12, atol=0)
    np.testing.assert_allclose(host(om)[idx], oo, rtol=1e-11, atol=1e-13 * np.abs(oo).max())
    np.testing.assert_allclose(host(Yb)[idx], yo, rtol=0, atol=1e-15)
    announce(f"PaSR {which}: {n} cells, {idx.size} sampled, kappa in [{ko.min():.3f}, {ko.max():.3f}]")
