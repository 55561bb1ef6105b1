"""The DI advance without allocation (chemk_advance_noalloc) against
chemk_advance on the same cells: two calls in a row, the second on fewer
cells, each bitwise equal to the allocating entry point's result; sizes above
the stated maximum and other modes are refused."""
import numpy as np
import pytest

from synth import mechanism as sm, workload as sw
from tests.gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu


def _both(ctx, T, p, Y, dt, opts):
    import torch
    n = T.size
    out = []
    for fn in (ctx.advance, ctx.advance_noalloc):
        Tt, Yt = dev(T), dev(np.ascontiguousarray(Y))
        st = torch.full((n,), -1, dtype=torch.int32, device="cuda:0")
        ns = torch.full((n,), -1, dtype=torch.int32, device="cuda:0")
        fn(Tt, dev(p), Yt, dt, st, ns, opts=opts)
        out.append((host(Tt), host(Yt), host(st), host(ns), ctx.last_counters()))
    return out


def test_noalloc_matches_advance_on_two_calls():
    from paper_2402_18858_amd import chemk
    mech = sm.mech_medium()
    ctx = chemk.Context(mech)
    T0, p0, Y0, _ = sw.flame_block(mech, 32, 2004)
    opts = chemk.default_opts(bins=16, waves_per_cu=8)
    for n in (20000, 3001):
        (Ta, Ya, sa, na, ca), (Tb, Yb, sb, nb, cb) = _both(ctx, T0[:n], p0[:n], Y0[:n], 5e-7, opts)
        announce(f"noalloc: {n} cells, steps {na.sum()} vs {nb.sum()}, counters {ca} vs {cb}")
        assert (sa == 0).all()
        assert np.array_equal(Ta, Tb) and np.array_equal(Ya, Yb)
        assert np.array_equal(sa, sb) and np.array_equal(na, nb)
        assert ca == cb
    # refused: above the maximum, ANN mode
    import torch
    big = chemk.lib.CHEMK_NOALLOC_MAX_CELLS if hasattr(chemk.lib, "CHEMK_NOALLOC_MAX_CELLS") else 262144
    Tt = torch.zeros(big + 1, dtype=torch.float64, device="cuda:0")
    Yt = torch.zeros((big + 1, mech.K), dtype=torch.float64, device="cuda:0")
    st = torch.zeros(big + 1, dtype=torch.int32, device="cuda:0")
    with pytest.raises(chemk.ChemkError) as ei:
        ctx.advance_noalloc(Tt, Tt, Yt, 5e-7, st, opts=opts)
    assert ei.value.code == chemk.E_ARG
    with pytest.raises(chemk.ChemkError) as ei:
        ctx.advance_noalloc(Tt[:10], Tt[:10], Yt[:10], 5e-7, st[:10],
                            opts=chemk.default_opts(mode=chemk.MODE_ANN))
    assert ei.value.code == chemk.E_ARG
