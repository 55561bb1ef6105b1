"""Parity of the GPU direct integration (DI) with the FP64 oracle.

Bar (the acceptance criteria of the chemistry advance): relative 1e-6 on
every Y_k above 1e-8 and 1e-4 K on T; element masses conserved to 1e-12
relative.  The oracle's results are precomputed by
tests/golden/make_golden.py (oracle only) at rtol 1e-10."""
import os

import numpy as np
import pytest

import oracle
from synth import mechanism as sm, workload as sw
from tests.gpu_util import announce, dev, element_mass, host

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _parity(Yg, Tg, Yo, To, ytol=1e-6, ttol=1e-4):
    mask = Yo > 1e-8
    rel = np.abs(Yg - Yo)[mask] / Yo[mask]
    dT = np.abs(Tg - To)
    return rel.max(), dT.max()


def _conservation(mech, Yin, Yout):
    m0 = element_mass(mech, Yin)
    m1 = element_mass(mech, Yout)
    return (np.abs(m1 - m0) / np.maximum(m0, 1e-300))[m0 > 1e-12].max()


def _run(ctx, T, p, Y, dt, **kw):
    import torch
    from paper_2402_18858_amd import chemk
    n = len(T)
    Tt, Yt = dev(T), dev(Y)
    st = torch.full((n,), -1, dtype=torch.int32, device="cuda:0")
    ns = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    ctx.advance(Tt, dev(p), Yt, dt, st, ns, opts=chemk.default_opts(**kw))
    return host(Tt), host(Yt), host(st), host(ns)


@pytest.fixture(scope="module")
def small_ctx():
    from paper_2402_18858_amd import chemk
    mech = sm.mech_small()
    return mech, chemk.Context(mech)


def test_di_probe_small(small_ctx):
    """16 cells with a bounded step budget: reports time and step counts first."""
    import time
    mech, ctx = small_ctx
    T, p, Y = sw.uniform_cells(mech, 16, 2001)
    announce("di probe: 16 small cells, max_steps 4000")
    t0 = time.time()
    Tg, Yg, st, ns = _run(ctx, T, p, Y, 1e-6, max_steps=4000)
    announce(f"di probe: {time.time() - t0:.3f} s, status {np.unique(st)}, steps {ns.tolist()}")
    assert (st == 0).all()


def test_di_small_full_parity(small_ctx):
    mech, ctx = small_ctx
    g = np.load(os.path.join(GOLD, "di_small_4096.npz"))
    T, p, Y = sw.uniform_cells(mech, 4096, 2001)
    announce("di small 4096 cells")
    Tg, Yg, st, ns = _run(ctx, T, p, Y, 1e-6)
    assert (g["status"] == 0).all()
    assert (st == 0).all(), np.unique(st, return_counts=True)
    ry, dT = _parity(Yg, Tg, g["Y"], g["T"])
    announce(f"small: max rel Y {ry:.3e}, max |dT| {dT:.3e} K, mean steps {ns.mean():.0f}")
    assert ry < 1e-6 and dT < 1e-4
    assert _conservation(mech, Y, Yg) < 1e-12


def test_di_small_tight_tolerance_matches_oracle_closely(small_ctx):
    mech, ctx = small_ctx
    g = np.load(os.path.join(GOLD, "di_small_4096.npz"))
    T, p, Y = sw.uniform_cells(mech, 4096, 2001)
    sel = np.arange(0, 4096, 16)
    Tg, Yg, st, ns = _run(ctx, T[sel], p[sel], Y[sel], 1e-6, rtol=1e-10, atol_Y=1e-18,
                          atol_T=1e-8)
    assert (st == 0).all()
    ry, dT = _parity(Yg, Tg, g["Y"][sel], g["T"][sel])
    announce(f"small rtol 1e-10: max rel Y {ry:.3e}, |dT| {dT:.3e}")
    assert ry < 1e-8 and dT < 1e-6


def test_di_results_independent_of_batching(small_ctx):
    """Bins, residency and graph capture change only the order cells are
    processed in: results must be bitwise identical."""
    mech, ctx = small_ctx
    T, p, Y = sw.uniform_cells(mech, 300, 77)
    ref = _run(ctx, T, p, Y, 1e-6, bins=1, waves_per_cu=4)
    for kw in (dict(bins=32, waves_per_cu=8), dict(bins=7, waves_per_cu=1, use_graph=1),
               dict(bins=16, use_graph=1)):
        out = _run(ctx, T, p, Y, 1e-6, **kw)
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), kw
        assert np.array_equal(out[2], ref[2]) and np.array_equal(out[3], ref[3])


def test_di_graph_replays(small_ctx):
    """A captured step replayed several times with eager work in between."""
    import torch
    from paper_2402_18858_amd import chemk
    mech, ctx = small_ctx
    T, p, Y = sw.uniform_cells(mech, 200, 78)
    ref = _run(ctx, T, p, Y, 1e-6)
    Tt, Yt, pt = dev(T), dev(Y), dev(p)
    st = torch.zeros(200, dtype=torch.int32, device="cuda:0")
    o = chemk.default_opts(use_graph=1)
    for rep in range(3):
        Tt.copy_(dev(T))
        Yt.copy_(dev(Y))
        torch.cuda.synchronize()
        ctx.advance(Tt, pt, Yt, 1e-6, st, None, opts=o)
        assert np.array_equal(host(Tt), ref[0]) and np.array_equal(host(Yt), ref[1]), rep
        _ = (torch.ones(1000, device="cuda:0") * 2).sum().item()   # eager work in between


def test_di_edge_cases(small_ctx):
    import torch
    from paper_2402_18858_amd import chemk
    mech, ctx = small_ctx
    T, p, Y = sw.uniform_cells(mech, 97, 79)
    # n = 0 is a no-op
    ctx.advance(dev(T[:0]), dev(p[:0]), dev(Y[:0]), 1e-6,
                torch.zeros(0, dtype=torch.int32, device="cuda:0"))
    # single cell equals the same cell inside a ragged batch
    one = _run(ctx, T[5:6], p[5:6], Y[5:6], 1e-6)
    many = _run(ctx, T, p, Y, 1e-6)
    assert np.array_equal(one[1][0], many[1][5]) and one[0][0] == many[0][5]
    # max_steps = 1: every cell fails with status 1 and keeps its input state
    Tg, Yg, st, ns = _run(ctx, T, p, Y, 1e-6, max_steps=1)
    assert (st == chemk.CELL_MAX_STEPS).all()
    assert np.array_equal(Tg, T) and np.array_equal(Yg, Y)
    # a non-finite cell is reported and does not disturb the others
    T2 = T.copy()
    T2[10] = np.nan
    Tg, Yg, st, ns = _run(ctx, T2, p, Y, 1e-6)
    assert st[10] != 0
    keep = np.arange(97) != 10
    assert np.array_equal(Yg[keep], many[1][keep])
    # argument errors are caught on the host, nothing enqueued
    with pytest.raises(chemk.ChemkError) as ei:
        ctx.advance(dev(T), dev(p), dev(Y), -1.0, torch.zeros(97, dtype=torch.int32,
                                                              device="cuda:0"))
    assert ei.value.code == chemk.E_ARG
    with pytest.raises(chemk.ChemkError):
        ctx.advance(dev(T), dev(p), dev(Y), 1e-6, torch.zeros(97, dtype=torch.int32,
                                                              device="cuda:0"),
                    opts=chemk.default_opts(rtol=0.0))
    # ANN mode before set-up is a state error
    with pytest.raises(chemk.ChemkError) as ei:
        ctx.advance(dev(T), dev(p), dev(Y), 1e-6, torch.zeros(97, dtype=torch.int32,
                                                              device="cuda:0"),
                    opts=chemk.default_opts(mode=chemk.MODE_ANN))
    assert ei.value.code == chemk.E_STATE


def test_di_medium_block_parity_at_full_size():
    """The full 64^3 block (262,144 cells, 32 species) in the launch
    configuration the benchmark times; oracle values on a stratified sample."""
    from paper_2402_18858_amd import chemk
    mech = sm.mech_medium()
    ctx = chemk.Context(mech)
    g = np.load(os.path.join(GOLD, "di_medium_sample.npz"))
    T, p, Y, region = sw.flame_block(mech, 64, 2002)
    announce("di medium 262144 cells")
    Tg, Yg, st, ns = _run(ctx, T, p, Y, 5e-7, use_graph=1)
    idx = g["idx"]
    assert (st == 0).all(), np.unique(st, return_counts=True)
    ry, dT = _parity(Yg[idx], Tg[idx], g["Y"], g["T"])
    announce(f"medium: max rel Y {ry:.3e}, |dT| {dT:.3e} K, mean steps {ns.mean():.1f}")
    assert ry < 1e-6 and dT < 1e-4
    assert _conservation(mech, Y, Yg) < 1e-12


@pytest.mark.parametrize("which", ["small", "medium"])
def test_di_register_lu_equals_lds_lu(which):
    """The register-resident LU (N = 10, 33) and the LDS LU factorise the
    same matrix with the same operations: the advance must agree bitwise,
    step counts and status included."""
    from paper_2402_18858_amd import chemk
    mech = getattr(sm, f"mech_{which}")()
    ctx = chemk.Context(mech)
    if which == "small":
        T, p, Y = sw.uniform_cells(mech, 300, 79)
        dt = 1e-6
    else:
        T, p, Y, region = sw.flame_block(mech, 16, 2003 if which == "medium" else 2006)
        keep = np.concatenate([np.nonzero(region == r)[0][:100 if which == "large" else 400]
                               for r in range(3)])
        T, p, Y = T[keep], p[keep], np.ascontiguousarray(Y[keep])
        dt = 5e-7
    announce(f"register LU vs LDS LU: {which}, {T.size} cells")
    a = _run(ctx, T, p, Y, dt, di_kernel=chemk.DI_LDS_LU)
    b = _run(ctx, T, p, Y, dt, di_kernel=chemk.DI_REG_LU)
    c = _run(ctx, T, p, Y, dt)
    assert (a[2] == 0).all(), np.unique(a[2], return_counts=True)
    for x, y_ in zip(a, b):
        assert np.array_equal(x, y_)
    for x, y_ in zip(b, c):
        assert np.array_equal(x, y_)
    announce(f"register LU vs LDS LU: {which} bitwise equal, mean steps {a[3].mean():.1f}")


@pytest.mark.parametrize("which", ["tiny", "large"])
def test_di_register_lu_unavailable_size_is_an_argument_error(which):
    """Mechanisms whose N has no register instance (5 species; 53, whose
    instance is switched off): auto falls back to the LDS LU, an explicit
    request is CHEMK_E_ARG."""
    from paper_2402_18858_amd import chemk
    from tests import mechs
    mech = mechs.tiny_hox() if which == "tiny" else sm.mech_large()
    ctx = chemk.Context(mech)
    n = 8
    T = np.full(n, 1500.0)
    p = np.full(n, 101325.0)
    Y = np.full((n, mech.K), 1.0 / mech.K)
    a = _run(ctx, T, p, Y, 1e-7, di_kernel=chemk.DI_LDS_LU)
    b = _run(ctx, T, p, Y, 1e-7)
    for x, y_ in zip(a, b):
        assert np.array_equal(x, y_)
    with pytest.raises(chemk.ChemkError) as e:
        _run(ctx, T, p, Y, 1e-7, di_kernel=chemk.DI_REG_LU)
    assert e.value.code == chemk.E_ARG


def test_autotune_cache_and_factorisation_axis(tmp_path, monkeypatch):
    """The autotuner also chooses the factorisation, caches its choice per
    (arch, CUs, K, R, E, log2 n) for the process and in CHEMK_TUNE_CACHE, and
    a cached key is answered without running DI."""
    import time
    from paper_2402_18858_amd import chemk
    mech = sm.mech_medium()
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("CHEMK_TUNE_CACHE", str(path))
    chemk.tune_cache_clear()
    T, p, Y, _ = sw.flame_block(mech, 16, 2004)
    Td, pd, Yd = dev(T), dev(p), dev(Y)
    ctx = chemk.Context(mech)
    t0 = time.time()
    b1 = ctx.autotune(Td, pd, Yd, 5e-7)
    t1 = time.time() - t0
    tun = ctx.tuning()
    assert tun[:2] == b1[:2] and tun[2] in (chemk.DI_AUTO, chemk.DI_LDS_LU)
    fields = path.read_text().split()
    assert len(fields) == 10 and fields[0].startswith("gfx950")
    assert [int(v) for v in fields[6:9]] == list(tun)
    announce(f"autotune: bins {tun[0]}, waves/CU {tun[1]}, factorisation {tun[2]} in {t1:.2f} s")
    ctx2 = chemk.Context(mech)
    t0 = time.time()
    b2 = ctx2.autotune(Td, pd, Yd, 5e-7)
    t2 = time.time() - t0
    assert b2 == b1 and ctx2.tuning() == tun
    assert t2 < 0.5 * t1, (t1, t2)
    # an emptied process cache is refilled from the file
    chemk.tune_cache_clear()
    ctx3 = chemk.Context(mech)
    b3 = ctx3.autotune(Td, pd, Yd, 5e-7)
    assert b3[:2] == b1[:2] and ctx3.tuning() == tun
    # the tuned context's advance equals one with the choice spelled out
    a = _run(ctx3, T, p, Y, 5e-7)
    c = _run(ctx3, T, p, Y, 5e-7, bins=tun[0], waves_per_cu=tun[1],
             di_kernel=tun[2] if tun[2] else chemk.DI_REG_LU)
    for x, y_ in zip(a, c):
        assert np.array_equal(x, y_)
    monkeypatch.delenv("CHEMK_TUNE_CACHE")
    chemk.tune_cache_clear()


def test_di_takes_the_oracles_steps():
    """The GPU integrator is the oracle's algorithm: on 384 flame-block cells
    (a third from each region) both run RODAS at the same tolerances from the
    same first step, so they accept and reject the same steps.  Step counts
    agree cell by cell (an accept/reject decision can only flip where the
    error estimate sits within rounding of 1), and the states agree far
    below the parity bar (both carry the same truncation error)."""
    from paper_2402_18858_amd import chemk
    mech = sm.mech_medium()
    ctx = chemk.Context(mech)
    T0, p0, Y0, region = sw.flame_block(mech, 32, 2004)
    rng = np.random.default_rng(5)
    idx = np.sort(np.concatenate([rng.choice(np.nonzero(region == r)[0], 128, replace=False) for r in range(3)]))
    T, p, Y = T0[idx], p0[idx], np.ascontiguousarray(Y0[idx])
    o = chemk.default_opts(rtol=1e-7)
    Tg, Yg, st, ns = _run(ctx, T, p, Y, 5e-7, rtol=o.rtol)
    To, Yo, so, nso = oracle.OracleMech(mech).advance(T, p, Y, 5e-7, rtol=o.rtol, atol_Y=o.atol_Y, atol_T=o.atol_T,
                                                      h0_frac=o.h0_frac, max_steps=o.max_steps)
    same = (ns == nso).mean()
    d = np.abs(ns.astype(np.int64) - nso)
    ry, dT = _parity(Yg, Tg, Yo, To)
    announce(f"steps vs the oracle's: {same * 100:.1f} % of cells equal, max |diff| {d.max()} of "
             f"{nso.max()}, means {ns.mean():.2f} / {nso.mean():.2f}; max rel Y {ry:.2e}, |dT| {dT:.2e} K")
    assert (st == 0).all() and (so == 0).all()
    assert same >= 0.98
    assert np.all(d <= np.maximum(2, 0.02 * nso))
    assert abs(ns.mean() - nso.mean()) <= 0.005 * nso.mean()
    assert ry < 1e-8 and dT < 1e-6
