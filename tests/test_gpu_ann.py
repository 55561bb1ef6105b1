"""The learned part on the GPU: forward, gradients and Adam against the FP64
oracle of the network (identical BF16 quantisation points), element
conservation of the projected ANN advance, and the trained network's gain
over frozen chemistry, judged by DI."""
import numpy as np
import pytest

from oracle import ann as oann
from synth import mechanism as sm, workload as sw
from tests.gpu_util import announce, dev, element_mass, host

pytestmark = pytest.mark.gpu

DIMS_SMALL = None


def _ctx_small_net(mech, seed=5):
    from paper_2402_18858_amd import chemk, train
    ctx = chemk.Context(mech)
    K = mech.K
    dims = [K + 2, 128, 64, K]
    ctx.ann_create(dims)
    params = train.init_params(dims, seed)
    rng = np.random.default_rng(seed)
    # non-zero biases so that their gradients and the bias path are exercised
    off = 0
    for i in range(len(dims) - 1):
        off += dims[i] * dims[i + 1]
        params[off:off + dims[i + 1]] = rng.normal(0, 0.1, dims[i + 1]).astype(np.float32)
        off += dims[i + 1]
    ctx.ann_set_weights(params)
    return ctx, dims, params


def _unpack(params, dims):
    Ws, bs, off = [], [], 0
    for i in range(len(dims) - 1):
        n = dims[i] * dims[i + 1]
        Ws.append(params[off:off + n].reshape(dims[i], dims[i + 1]).astype(np.float64))
        off += n
        bs.append(params[off:off + dims[i + 1]].astype(np.float64))
        off += dims[i + 1]
    return Ws, bs


def _states(mech, n, seed):
    T, p, Y = sw.uniform_cells(mech, n, seed, T_range=(600, 2400))
    return T, p, Y


def _oracle_inputs(T, p, Y, mu_x, sd_x):
    return (oann.raw_features(T, p, Y) - mu_x) / sd_x


def _set_norm(ctx, mech, T, p, Y):
    F, K = mech.K + 2, mech.K
    raw = oann.raw_features(T, p, Y)
    mu_x, sd_x = oann.norm_stats(raw)
    mu_y, sd_y = np.zeros(K), np.full(K, 1e-3)
    ctx.ann_set_norm(mu_x, sd_x, mu_y, sd_y, 5e-7)
    return mu_x, sd_x


def test_forward_matches_oracle():
    import torch
    mech = sm.mech_medium()
    ctx, dims, params = _ctx_small_net(mech)
    T, p, Y = _states(mech, 333, 41)      # ragged: not a multiple of the 128-row tile
    mu_x, sd_x = _set_norm(ctx, mech, T, p, Y)
    X = torch.empty((333, 64), dtype=torch.int16, device="cuda:0")
    ctx.ann_pack(dev(T), dev(p), dev(Y), None, X, None)
    out = torch.empty((333, mech.K), dtype=torch.float32, device="cuda:0")
    ctx.ann_forward_packed(X, out)
    g = host(out).astype(np.float64)
    Ws, bs = _unpack(params, dims)
    o, _ = oann.forward(Ws, bs, _oracle_inputs(T, p, Y, mu_x, sd_x), quantize=True)
    rel_rms = np.sqrt(np.mean((g - o) ** 2)) / np.sqrt(np.mean(o ** 2))
    announce(f"forward: rel rms {rel_rms:.2e}, max abs {np.abs(g - o).max():.2e} = "
             f"{np.abs(g - o).max() / o.std():.2e} of the outputs' spread")
    assert rel_rms < 2e-3
    assert np.abs(g - o).max() < 1e-2 * o.std()


@pytest.mark.parametrize("n,hidden", [(777, None), (1024, None), (777, (1024, 512, 192)),
                                      (1024, (960, 512, 256))])
def test_forward_full_network_matches_oracle(n, hidden):
    """The production network (34-1024-512-256-32) against the oracle network,
    on a row count ragged against the GEMM tile (777: the last row block takes
    the bounds-checked epilogue) and on one the 128-row tiles divide (1,024:
    every tile takes the epilogue staged through LDS); hidden widths
    1024-512-192, which give the direct-to-LDS kernel a partial column tile
    (layer 3, N = 192) and the register-ring kernel a K of three slabs
    (layer 4); and 960-512-256, which give the one-slab first layer a partial
    column tile (N = 960) and the register-ring kernel K = 960 (15 slabs)."""
    import torch
    from paper_2402_18858_amd import chemk, train
    mech = sm.mech_medium()
    ctx = chemk.Context(mech)
    dims = train.default_dims(mech.K) if hidden is None else [mech.K + 2, *hidden, mech.K]
    ctx.ann_create(dims)
    params = train.init_params(dims, 21)
    rng = np.random.default_rng(21)
    off = 0
    for i in range(len(dims) - 1):
        off += dims[i] * dims[i + 1]
        params[off:off + dims[i + 1]] = rng.normal(0, 0.1, dims[i + 1]).astype(np.float32)
        off += dims[i + 1]
    ctx.ann_set_weights(params)
    T, p, Y = _states(mech, n, 45)
    mu_x, sd_x = _set_norm(ctx, mech, T, p, Y)
    X = torch.empty((n, 64), dtype=torch.int16, device="cuda:0")
    ctx.ann_pack(dev(T), dev(p), dev(Y), None, X, None)
    out = torch.empty((n, mech.K), dtype=torch.float32, device="cuda:0")
    ctx.ann_forward_packed(X, out)
    g = host(out).astype(np.float64)
    Ws, bs = _unpack(params, dims)
    o, _ = oann.forward(Ws, bs, _oracle_inputs(T, p, Y, mu_x, sd_x), quantize=True)
    rel_rms = np.sqrt(np.mean((g - o) ** 2)) / np.sqrt(np.mean(o ** 2))
    announce(f"forward (network {dims}, {n} rows): rel rms {rel_rms:.2e}, max abs "
             f"{np.abs(g - o).max():.2e} = {np.abs(g - o).max() / o.std():.2e} of the outputs' spread")
    assert rel_rms < 2e-3
    assert np.abs(g - o).max() < 1e-2 * o.std()


def test_gradients_match_oracle():
    import torch
    mech = sm.mech_medium()
    ctx, dims, params = _ctx_small_net(mech, seed=6)
    B = 192
    T, p, Y = _states(mech, B, 42)
    mu_x, sd_x = _set_norm(ctx, mech, T, p, Y)
    rng = np.random.default_rng(7)
    Zt = rng.normal(0, 1, (B, mech.K)).astype(np.float32)
    X = torch.empty((B, 64), dtype=torch.int16, device="cuda:0")
    ctx.ann_pack(dev(T), dev(p), dev(Y), None, X, None)
    idx = dev(np.arange(B, dtype=np.int32))
    grads = torch.zeros(ctx.ann_param_count(), dtype=torch.float32, device="cuda:0")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    ctx.ann_train_step(idx, X, dev(Zt), 0.0, update=False, loss=loss, grads=grads)
    gg = host(grads).astype(np.float64)
    Ws, bs = _unpack(params, dims)
    o, cache = oann.forward(Ws, bs, _oracle_inputs(T, p, Y, mu_x, sd_x), quantize=True)
    lo, dout = oann.mse_loss(o, Zt.astype(np.float64))
    gW, gb = oann.backward(Ws, bs, cache, dout, quantize=True)
    ref = np.concatenate([np.concatenate([w.ravel(), b]) for w, b in zip(gW, gb)])
    rel = np.sqrt(np.mean((gg - ref) ** 2)) / np.sqrt(np.mean(ref ** 2))
    announce(f"gradients: rel rms {rel:.2e}; loss gpu {host(loss)[0]:.6f} oracle {lo:.6f}")
    assert host(loss)[0] == pytest.approx(lo, rel=1e-3)
    assert rel < 1e-2
    # per layer as well
    off = 0
    for i, (w, b) in enumerate(zip(gW, gb)):
        seg = gg[off:off + w.size + b.size]
        r = np.concatenate([w.ravel(), b])
        off += w.size + b.size
        assert np.sqrt(np.mean((seg - r) ** 2)) < 2e-2 * np.sqrt(np.mean(r ** 2)), i


def test_hrr_weights_match_oracle():
    """Eq. 10's heat-release weights and scale computed on the device."""
    import torch
    import oracle
    mech = sm.mech_medium()
    ctx, dims, params = _ctx_small_net(mech, seed=10)
    n = 300
    T, p, Y = _states(mech, n, 46)
    _set_norm(ctx, mech, T, p, Y)
    rng = np.random.default_rng(11)
    dY = rng.normal(0, 1e-4, Y.shape)
    dY -= dY.mean(1, keepdims=True)
    G = torch.zeros((n, mech.K), dtype=torch.float32, device="cuda:0")
    s = ctx.ann_hrr_weights(dev(T), dev(p), dev(Y), dev(Y + dY), 5e-7, G)
    om = oracle.OracleMech(mech)
    Go, so, _ = oann.hrr_label_weights(om.species_thermo, om.W, T, p, Y, Y + dY, 5e-7, np.full(mech.K, 1e-3))
    g = host(G).astype(np.float64)
    announce(f"hrr weights: scale {s:.6e} (oracle {so:.6e}), max rel dG {np.abs(g - Go).max() / np.abs(Go).max():.2e}")
    assert s == pytest.approx(so, rel=1e-10)
    np.testing.assert_allclose(g, Go, rtol=1e-6, atol=1e-7 * np.abs(Go).max())
    # a given scale is used as is
    G2 = torch.zeros_like(G)
    s2 = ctx.ann_hrr_weights(dev(T), dev(p), dev(Y), None, 5e-7, G2, scale=2.0 * so)
    assert s2 == 2.0 * so
    np.testing.assert_allclose(host(G2).astype(np.float64), Go / 2.0, rtol=1e-6, atol=1e-7 * np.abs(Go).max())


def test_physics_loss_gradients_match_oracle():
    """Eq. 11 with the mass (Eq. 9) and heat-release (Eq. 10) terms: loss and
    gradients of one step against the oracle."""
    import torch
    mech = sm.mech_medium()
    ctx, dims, params = _ctx_small_net(mech, seed=12)
    B = 256
    T, p, Y = _states(mech, B, 47)
    mu_x, sd_x = _set_norm(ctx, mech, T, p, Y)
    rng = np.random.default_rng(13)
    Zt = rng.normal(0, 1, (B, mech.K)).astype(np.float32)
    Gh = rng.normal(0, 0.3, (B, mech.K)).astype(np.float32)
    X = torch.empty((B, 64), dtype=torch.int16, device="cuda:0")
    ctx.ann_pack(dev(T), dev(p), dev(Y), None, X, None)
    idx = dev(rng.permutation(B).astype(np.int32))
    grads = torch.zeros(ctx.ann_param_count(), dtype=torch.float32, device="cuda:0")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    wm, wh = 0.5, 0.25
    ctx.ann_train_step(idx, X, dev(Zt), 0.0, update=False, loss=loss, grads=grads, G=dev(Gh), w_mass=wm,
                       w_hrr=wh)
    gg = host(grads).astype(np.float64)
    order = host(idx)
    Ws, bs = _unpack(params, dims)
    o, cache = oann.forward(Ws, bs, _oracle_inputs(T, p, Y, mu_x, sd_x)[order], quantize=True)
    lo, dout = oann.phys_loss(o, Zt[order].astype(np.float64), np.zeros(mech.K), np.full(mech.K, 1e-3),
                              Gh[order].astype(np.float64), wm, wh)
    gW, gb = oann.backward(Ws, bs, cache, dout, quantize=True)
    ref = np.concatenate([np.concatenate([w.ravel(), b]) for w, b in zip(gW, gb)])
    rel = np.sqrt(np.mean((gg - ref) ** 2)) / np.sqrt(np.mean(ref ** 2))
    lo_data, _ = oann.mse_loss(o, Zt[order].astype(np.float64))
    announce(f"physics-loss gradients: rel rms {rel:.2e}; loss gpu {host(loss)[0]:.6f} oracle {lo:.6f} "
             f"(data term {lo_data:.6f})")
    assert host(loss)[0] == pytest.approx(lo, rel=1e-3)
    assert rel < 1e-2
    with pytest.raises(Exception):
        ctx.ann_train_step(idx, X, dev(Zt), 0.0, update=False, w_hrr=0.5)   # G missing


def test_adam_step_matches_oracle():
    import torch
    mech = sm.mech_medium()
    ctx, dims, params = _ctx_small_net(mech, seed=8)
    B = 128
    T, p, Y = _states(mech, B, 43)
    mu_x, sd_x = _set_norm(ctx, mech, T, p, Y)
    Zt = np.random.default_rng(9).normal(0, 1, (B, mech.K)).astype(np.float32)
    X = torch.empty((B, 64), dtype=torch.int16, device="cuda:0")
    ctx.ann_pack(dev(T), dev(p), dev(Y), None, X, None)
    ctx.ann_reset_optimizer()
    lr = 1e-3
    ctx.ann_train_step(dev(np.arange(B, dtype=np.int32)), X, dev(Zt), lr, update=True)
    new = ctx.ann_get_weights().astype(np.float64)
    Ws, bs = _unpack(params, dims)
    o, cache = oann.forward(Ws, bs, _oracle_inputs(T, p, Y, mu_x, sd_x), quantize=True)
    _, dout = oann.mse_loss(o, Zt.astype(np.float64))
    gW, gb = oann.backward(Ws, bs, cache, dout, quantize=True)
    g = np.concatenate([np.concatenate([w.ravel(), b]) for w, b in zip(gW, gb)])
    p0 = params.astype(np.float64)
    p1, _, _ = oann.adam_step(p0, g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    # first Adam step moves each weight by about lr * sign(g); compare where
    # the gradient is well above the rounding noise of the two evaluations
    big = np.abs(g) > 1e-3 * np.abs(g).max()
    d = np.abs((new - p0) - (p1 - p0))[big]
    announce(f"adam: {big.sum()} params compared, max |diff| {d.max():.2e} (lr {lr})")
    assert d.max() < 1e-2 * lr + 1e-7


def _ratio_inside(mech, Y, ratios):
    """Element-ratio windows by their definition: z = element mass fractions,
    lo <= (num . z) / (den . z) <= hi with a positive denominator."""
    E = oann.element_matrix(mech.composition, mech.element_mass)
    z = Y @ E.T
    ok = np.ones(Y.shape[0], bool)
    for num, den, lo, hi in ratios:
        u, d = z @ num, z @ den
        ok &= (d > 0) & (u >= lo * d) & (u <= hi * d)
    return ok


def _expected_ann_step(mech, ctx, T, p, Y, out, checks, box):
    """The oracle's ANN step on the network output `out` (the GPU's own, so
    that the post step is compared alone): post_state, T from the conserved
    enthalpy, the routing decisions.  Returns (Y, T, routed, margin) where
    margin marks cells whose decisions sit within rounding of a bound."""
    import oracle
    mx, sx, my, sy, _ = ctx.ann_get_norm()
    lo, hi, neg_tol = box
    Emat = oann.element_matrix(mech.composition, mech.element_mass)
    dY = my + sy * out
    Yo, ok, adj = oann.post_state(Emat, Y, dY, sy, neg_tol=neg_tol)
    om = oracle.OracleMech(mech)
    _, h0 = om.thermo_batch(T, Y)
    To, sto = om.T_from_h_batch(h0, Yo, T)
    raw = oann.raw_features(T, p, Y)
    inside = np.all((raw >= lo) & (raw <= hi), 1) & _ratio_inside(mech, Y, checks["ratios"])
    dT = To - T
    dlo, dhi = checks["dT"]
    amax = checks["adj_max"] if checks["adj_max"] > 0 else np.inf
    routed = ~inside | ~ok | (adj > amax) | (sto != 0) | (dT < dlo) | (dT > dhi)
    margin = (np.abs(Yo.min(1) + neg_tol) <= 1e-13) | \
        (np.minimum(np.abs(dT - dlo), np.abs(dT - dhi)) <= 1e-7)
    if np.isfinite(amax):
        margin |= np.abs(adj - amax) <= 1e-9 * amax
    return Yo, To, routed, margin


def _run_ann(ctx, T, p, Y, dt, use_graph=0):
    import torch
    from paper_2402_18858_amd import chemk
    n = T.size
    Tt, Yt = dev(T), dev(Y)
    st = torch.full((n,), -1, dtype=torch.int32, device="cuda:0")
    ctx.advance(Tt, dev(p), Yt, dt, st, None,
                opts=chemk.default_opts(mode=chemk.MODE_ANN, use_graph=use_graph))
    return host(Tt), host(Yt), host(st)


def _gpu_out(ctx, T, p, Y):
    import torch
    n = T.size
    X = torch.empty((n, 64), dtype=torch.int16, device="cuda:0")
    ctx.ann_pack(dev(T), dev(p), dev(Y), None, X, None)
    out = torch.empty((n, ctx.K), dtype=torch.float32, device="cuda:0")
    ctx.ann_forward_packed(X, out)
    return host(out).astype(np.float64)


def _check_ann_step(mech, ctx, T, p, Y, Tg, Yg, sg, checks, what):
    """GPU ANN step against the oracle's post step on the GPU's network output,
    cell by cell: routing decisions (but for cells on a bound), Y of the
    network cells, T from the conserved enthalpy, element conservation."""
    from paper_2402_18858_amd import chemk
    lo, hi, neg_tol = ctx.ann_get_envelope()
    out = _gpu_out(ctx, T, p, Y)
    _, _, _, sy, _ = ctx.ann_get_norm()
    Yo, To, routed_o, margin = _expected_ann_step(mech, ctx, T, p, Y, out, checks, (lo, hi, neg_tol))
    routed = (sg & chemk.CELL_ROUTED_DI) != 0
    mism = (routed != routed_o) & ~margin
    net = ~routed & ~routed_o
    d = np.abs(Yg[net] - Yo[net])
    rel_sd = (d / sy[None, :]).max() if net.any() else 0.0
    announce(f"{what}: {T.size} cells, routed {routed.sum()} (oracle {routed_o.sum()}, "
             f"{margin.sum()} on a bound, {mism.sum()} disagree); network cells {net.sum()}: "
             f"max |dY| {d.max() if net.any() else 0:.2e} = {rel_sd:.2e} sd, "
             f"max |dT| {np.abs(Tg[net] - To[net]).max() if net.any() else 0:.2e} K")
    assert mism.sum() == 0, np.nonzero(mism)[0][:10]
    assert (sg[net] == 0).all()
    # FP64 on both sides: the agreement is far below the spread sd_k, down to
    # the rounding of Y itself for species whose spread is at its floor
    if net.any():
        assert (d <= 1e-8 * sy[None, :] + 2e-15).all()
    assert np.abs(Tg[net] - To[net]).max() < 1e-8 * T.max()
    assert Yg[net].min() >= -neg_tol
    m0, m1 = element_mass(mech, Y[net]), element_mass(mech, Yg[net])
    assert (np.abs(m1 - m0) / np.maximum(m0, 1e-300))[m0 > 1e-12].max() < 1e-12
    return routed, net


def test_ann_advance_matches_oracle_post_step():
    """ANN mode of chemk_advance against the oracle's post step: the prediction
    corrected to the input's element masses in units of each species' spread
    sd_k (weights sd^2, spreads spanning three decades here), negatives held at
    zero over up to four solves, T from the conserved enthalpy, and the output
    checks (correction limit, dT window) deciding which cells go to DI.  The
    oracle runs on the GPU's own network output, so that the post step is
    compared alone (the network has its own tests).  Random weights drive many
    absent species negative, so the active set is exercised on most cells."""
    mech = sm.mech_medium()
    ctx, dims, params = _ctx_small_net(mech, seed=11)
    n = 1000
    T, p, Y = _states(mech, n, 44)
    Y[:300, :8] = 0.0                              # absent species, as in cold cells
    Y /= Y.sum(1, keepdims=True)
    raw = oann.raw_features(T, p, Y)
    mu_x, sd_x = oann.norm_stats(raw)
    rng = np.random.default_rng(12)
    sd_y = 10.0 ** rng.uniform(-5.5, -2.5, mech.K)
    ctx.ann_set_norm(mu_x, sd_x, np.zeros(mech.K), sd_y, 5e-7)
    ctx.ann_set_checks(adj_max=2.5, dT=(-40.0, 60.0))
    checks = ctx.ann_get_checks()
    Tg, Yg, sg = _run_ann(ctx, T, p, Y, 5e-7)
    out = _gpu_out(ctx, T, p, Y)
    assert (Y + sd_y * out < 0).any(1).mean() > 0.3
    routed, net = _check_ann_step(mech, ctx, T, p, Y, Tg, Yg, sg, checks, "ann advance")
    assert 0.05 < routed.mean() < 0.95
    # the network against the oracle network (same BF16 rounding points)
    Ws, bs = _unpack(params, dims)
    o, _ = oann.forward(Ws, bs, _oracle_inputs(T, p, Y, mu_x, sd_x), quantize=True)
    rel_rms = np.sqrt(np.mean((out - o) ** 2)) / np.sqrt(np.mean(o ** 2))
    assert rel_rms < 2e-3
    assert np.abs(out - o).max() < 1e-2 * o.std()


def _trained_medium(ctx):
    from paper_2402_18858_amd import train
    return train.load(ctx)


def test_ann_step_multichunk_matches_oracle():
    """The production network (trained weights, 34-1024-512-256-32) on more
    cells than one MLP chunk holds (65,536): 65,536 + 4,097 flame-block cells,
    so the step runs two chunks and a ragged tail.  Sampled rows of the GPU's
    network output against the oracle network (1e-2 of the outputs' spread),
    and every cell's post step and routing against the oracle's post step."""
    from paper_2402_18858_amd import chemk, train
    mech = sm.mech_medium()
    ctx = chemk.Context(mech)
    _trained_medium(ctx)
    ck = ctx.ann_get_checks()
    ctx.ann_set_checks(adj_max=train.ADJ_MAX, dT=ck["dT"], ratios=ck["ratios"])
    T0, p0, Y0, _ = sw.flame_block(mech, 64, 2002)
    n = 65536 + 4097
    pick = np.random.default_rng(7).choice(T0.size, n, replace=False)
    T, p, Y = T0[pick].copy(), p0[pick].copy(), np.ascontiguousarray(Y0[pick])
    Tg, Yg, sg = _run_ann(ctx, T, p, Y, 5e-7)
    _check_ann_step(mech, ctx, T, p, Y, Tg, Yg, sg, ctx.ann_get_checks(), "multi-chunk ANN step")
    out = _gpu_out(ctx, T, p, Y)
    rows = np.unique(np.concatenate([np.arange(0, 64), np.arange(65536 - 64, 65536 + 64),
                                     np.arange(n - 64, n),
                                     np.random.default_rng(8).choice(n, 300, replace=False)]))
    d = np.load(__import__("paper_2402_18858_amd.train", fromlist=["WEIGHTS"]).WEIGHTS,
                allow_pickle=False)
    Ws, bs = _unpack(d["params"], [int(v) for v in d["dims"]])
    o, _ = oann.forward(Ws, bs, _oracle_inputs(T[rows], p[rows], Y[rows], d["mu_x"], d["sd_x"]),
                        quantize=True)
    g = out[rows]
    rel_rms = np.sqrt(np.mean((g - o) ** 2)) / np.sqrt(np.mean(o ** 2))
    announce(f"multi-chunk forward, {rows.size} sampled rows: rel rms {rel_rms:.2e}, max "
             f"{np.abs(g - o).max():.2e} (outputs' spread {o.std():.2e})")
    assert rel_rms < 2e-3
    # Max bar 5e-2 in the outputs' z-scored units (sd(dY) = 1).  Single
    # outputs of the trained network move by whole BF16 steps of hidden
    # activations that round the other way: a one-ulp change of the oracle's
    # own FP32 pre-activations already moves the largest of 64,000 outputs by
    # 1-2e-2, and the GPU's FP32 accumulation order and GELU polynomial flip
    # more activations than one ulp does (the random networks above stay
    # within 1e-2 of their spread).
    assert np.abs(g - o).max() < 5e-2


def test_ann_routed_cells_equal_plain_di():
    """Cells the envelope routes (here: T above the median, by a tightened T
    window) are advanced by DI inside the ANN step: status exactly
    CELL_ROUTED_DI and Y, T bitwise equal to a DI-mode advance of the same
    cells (whose accuracy the DI parity tests pin against the oracle)."""
    import torch
    from paper_2402_18858_amd import chemk
    mech = sm.mech_medium()
    ctx = chemk.Context(mech)
    _trained_medium(ctx)
    T0, p0, Y0, region = sw.flame_block(mech, 32, 2002)
    n = 3000
    pick = np.random.default_rng(9).choice(T0.size, n, replace=False)
    T, p, Y = T0[pick].copy(), p0[pick].copy(), np.ascontiguousarray(Y0[pick])
    lo, hi, nt = ctx.ann_get_envelope()
    hi = hi.copy()
    hi[mech.K] = np.median(T)
    ctx.ann_set_envelope(lo, hi, nt)
    Tg, Yg, sg = _run_ann(ctx, T, p, Y, 5e-7)
    hot = T > hi[mech.K]
    routed = (sg & chemk.CELL_ROUTED_DI) != 0
    assert routed[hot].all()
    idx = np.nonzero(routed)[0]
    assert idx.size >= n // 2 - 1
    assert (sg[idx] == chemk.CELL_ROUTED_DI).all(), np.unique(sg[idx])
    Td, Yd = dev(T[idx]), dev(np.ascontiguousarray(Y[idx]))
    sd = torch.full((idx.size,), -1, dtype=torch.int32, device="cuda:0")
    ctx.advance(Td, dev(p[idx]), Yd, 5e-7, sd, None, opts=chemk.default_opts())
    assert (host(sd) == 0).all()
    announce(f"routed cells: {idx.size} of {n}, DI in the step equals plain DI bitwise")
    assert np.array_equal(host(Td), Tg[idx])
    assert np.array_equal(host(Yd), Yg[idx])
    cnt = ctx.last_counters()
    assert cnt["routed"] == 0      # the last call was the plain DI advance


def test_ann_step_graph_replays_match_eager():
    """ANN mode with use_graph=1: every replay of the captured step equals the
    eager step bitwise, with eager work and synchronisations between the
    replays; after set_checks (new routing) and after a new network
    (ann_create + weights + norm), the next call captures a new graph and
    again equals the eager step."""
    from paper_2402_18858_amd import chemk, train
    mech = sm.mech_medium()
    ctx = chemk.Context(mech)
    _trained_medium(ctx)
    T0, p0, Y0, _ = sw.flame_block(mech, 32, 2003)
    n = 20000
    T, p, Y = T0[:n].copy(), p0[:n].copy(), np.ascontiguousarray(Y0[:n])
    import torch
    Pt = dev(p)
    Tt, Yt = dev(T), dev(Y)
    st = torch.full((n,), -1, dtype=torch.int32, device="cuda:0")
    og = chemk.default_opts(mode=chemk.MODE_ANN, use_graph=1)

    def graph_step():
        Tt.copy_(dev(T))
        Yt.copy_(dev(Y))
        st.fill_(-1)
        ctx.advance(Tt, Pt, Yt, 5e-7, st, None, opts=og)
        torch.cuda.synchronize()
        return host(Tt), host(Yt), host(st)

    for phase in range(3):
        ref = _run_ann(ctx, T, p, Y, 5e-7)
        for rep in range(3):
            got = graph_step()
            for a_, b_ in zip(ref, got):
                assert np.array_equal(a_, b_), (phase, rep)
            _run_ann(ctx, T[:500], p[:500], Y[:500], 5e-7)      # eager work in between
        nr = int(((ref[2] & chemk.CELL_ROUTED_DI) != 0).sum())
        announce(f"graph phase {phase}: 3 replays equal the eager step ({nr} routed)")
        if phase == 0:
            ck = ctx.ann_get_checks()
            ctx.ann_set_checks(adj_max=0.5, dT=ck["dT"], ratios=ck["ratios"])
        elif phase == 1:
            d = train.load(ctx)                                  # new network state
            ctx.ann_set_norm(d["mu_x"], d["sd_x"], d["mu_y"], 0.9 * d["sd_y"], float(d["dt"]))


def test_training_reduces_loss_and_beats_frozen_chemistry():
    """Small end-to-end run of the pipeline on the 9-species mechanism: DI
    labels on the GPU, training by the library's kernels, held-out error
    judged by DI; the trained network must be >= 10x better than frozen
    chemistry (dY = 0) in normalised RMS."""
    from paper_2402_18858_amd import chemk, train
    mech = sm.mech_small()
    ctx = chemk.Context(mech)
    announce("training: small mechanism pipeline")
    data = train.generate_pairs(ctx, mech, 1e-6, 60000, n_rec=60, t_end=0.5, log=announce)
    hist = train.train_network(ctx, data, 1e-6, epochs=80, batch=1024, log=announce, mech=mech)
    assert hist["loss"][-1] < 0.5 * hist["loss"][0]
    hold = hist["holdout_index"]
    T, p, Y, Yn = data[:4]
    ev = train.evaluate(ctx, T[hold], p[hold], Y[hold], Yn[hold])
    announce(f"held-out normalised RMS {ev['rms_norm_all']:.3e} vs frozen "
             f"{ev['frozen_rms_norm_all']:.3e}; per species {np.round(ev['rms_norm'], 4)}")
    assert ev["rms_norm_all"] * 10 <= ev["frozen_rms_norm_all"]


def test_ann_advance_conserves_elements_and_routes():
    """ANN mode of chemk_advance: projected predictions conserve element
    masses to 1e-12; cells outside the envelope are advanced by DI and
    flagged; dt other than the trained one is refused."""
    import torch
    from paper_2402_18858_amd import chemk, train
    mech = sm.mech_small()
    ctx = chemk.Context(mech)
    data = train.generate_pairs(ctx, mech, 1e-6, 20000, n_rec=40, t_end=0.5, log=announce)
    train.train_network(ctx, data, 1e-6, epochs=3, batch=1024, log=announce, mech=mech)
    # states of the training distribution (inside the envelope) ...
    pick = np.random.default_rng(2001).choice(data[0].size, 2000, replace=False)
    T, p, Y = data[0][pick].copy(), data[1][pick].copy(), np.ascontiguousarray(data[2][pick])
    T[:20] = 150.0                           # ... and 20 far outside it -> DI
    Tt, Yt = dev(T), dev(Y)
    st = torch.full((2000,), -1, dtype=torch.int32, device="cuda:0")
    ctx.advance(Tt, dev(p), Yt, 1e-6, st, None, opts=chemk.default_opts(mode=chemk.MODE_ANN))
    s = host(st)
    Yg = host(Yt)
    routed = (s & chemk.CELL_ROUTED_DI) != 0
    assert routed[:20].all()
    ok = s == 0
    assert ok.mean() > 0.5, np.unique(s, return_counts=True)
    m0, m1 = element_mass(mech, Y), element_mass(mech, Yg)
    rel = np.abs(m1 - m0) / np.maximum(m0, 1e-300)
    assert rel[ok][m0[ok] > 1e-12].max() < 1e-12
    cnt = ctx.last_counters()
    assert cnt["routed"] == int(routed.sum())
    with pytest.raises(chemk.ChemkError) as ei:
        ctx.advance(Tt, dev(p), Yt, 2e-6, st, None, opts=chemk.default_opts(mode=chemk.MODE_ANN))
    assert ei.value.code == chemk.E_DT


_M64 = (1 << 64) - 1


def _mix64(z):
    """SplitMix64's output function (Steele, Lea, Flood 2014)."""
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def _perm(i, n, half, key):
    """Four-round balanced Feistel permutation of [0, n) with cycle walking."""
    mask = (1 << half) - 1
    x = i
    while True:
        L, R = x >> half, x & mask
        for r in range(4):
            t = L ^ (_mix64((key + 0x9E3779B97F4A7C15 * (r + 1) + R) & _M64) & mask)
            L, R = R, t
        x = (L << half) | R
        if x < n:
            return x


def test_train_loop_matches_step_sequence():
    """chemk_ann_train (device-side shuffles, cosine schedule, Adam on device
    counters, one captured step replayed) against the same steps issued one
    by one through chemk_ann_train_step with the batch rows and learning rates
    computed here from their definitions; the epoch losses, the held-out loss
    against the network's output, and the eager loop against the graph."""
    import math

    import torch
    mech = sm.mech_medium()
    n, B, epochs, seed, lr0, lr1 = 1000, 128, 2, 77, 2e-3, 1e-4
    T, p, Y = _states(mech, n + 200, 46)
    Zt = np.random.default_rng(10).normal(0, 1, (n + 200, mech.K)).astype(np.float32)
    ctxs = []
    for _ in range(3):
        ctx, dims, params = _ctx_small_net(mech, seed=12)
        _set_norm(ctx, mech, T, p, Y)
        ctx.ann_reset_optimizer()
        ctxs.append(ctx)
    X = torch.empty((n + 200, 64), dtype=torch.int16, device="cuda:0")
    ctxs[0].ann_pack(dev(T), dev(p), dev(Y), None, X, None)
    Z = dev(Zt)
    Xt, Zs, Xh, Zh = X[:n].contiguous(), Z[:n].contiguous(), X[n:].contiguous(), Z[n:].contiguous()
    el, hl = ctxs[0].ann_train(Xt, Zs, epochs, batch=B, lr0=lr0, lr1=lr1, seed=seed, X_hold=Xh,
                               Z_hold=Zh, use_graph=True)
    el2, hl2 = ctxs[1].ann_train(Xt, Zs, epochs, batch=B, lr0=lr0, lr1=lr1, seed=seed, X_hold=Xh,
                                 Z_hold=Zh, use_graph=False)
    w0, w1 = ctxs[0].ann_get_weights(), ctxs[1].ann_get_weights()
    # same steps, same weights; the losses are sums of per-block atomics
    assert np.array_equal(w0, w1)
    assert np.allclose(el, el2, rtol=1e-6) and np.allclose(hl, hl2, rtol=1e-6)
    # the same steps one at a time
    spe = n // B
    total = spe * epochs
    half = 1
    while (1 << (2 * half)) < n:
        half += 1
    ref = ctxs[2]
    loss = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    losses = []
    for s in range(total):
        e, b = divmod(s, spe)
        key = _mix64(seed ^ _mix64(e + 1))
        idx = np.array([_perm(b * B + r, n, half, key) for r in range(B)], np.int32)
        if b == 0:
            seen = set()
        assert not seen.intersection(idx.tolist())
        seen.update(idx.tolist())
        lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * s / total))
        ref.ann_train_step(dev(idx), Xt, Zs, lr, update=True, loss=loss)
        losses.append(float(host(loss)[0]))
    wr = ref.ann_get_weights()
    ep_loss = np.array(losses).reshape(epochs, spe).mean(1)
    announce(f"train loop: {total} steps, max |w - w_steps| {np.abs(w0 - wr).max():.2e}, "
             f"epoch losses {el} vs {ep_loss}, held-out {hl}")
    assert np.abs(w0 - wr).max() <= 1e-6 * max(1.0, np.abs(wr).max())
    assert np.allclose(el, ep_loss, rtol=1e-5)
    out = torch.empty((200, mech.K), dtype=torch.float32, device="cuda:0")
    ctxs[0].ann_forward_packed(Xh, out)
    mse = np.mean((host(out).astype(np.float64) - Zt[n:]) ** 2)
    assert hl[-1] == pytest.approx(mse, rel=1e-5)


def test_training_in_schedule_slices_equals_one_call():
    """chemk_ann_train over 4 epochs in one call and as two calls of 2 epochs
    (epoch0 = 0, 2 of epochs_total = 4): the same learning rates, row orders
    and Adam step counts, so the same weights bitwise and the same epoch
    losses."""
    import torch
    mech = sm.mech_medium()
    outs = []
    for sliced in (False, True):
        ctx, dims, params = _ctx_small_net(mech, seed=14)
        n = 1024
        T, p, Y = _states(mech, n, 48)
        _set_norm(ctx, mech, T, p, Y)
        Zt = np.random.default_rng(15).normal(0, 1, (n, mech.K)).astype(np.float32)
        X = torch.empty((n, 64), dtype=torch.int16, device="cuda:0")
        ctx.ann_pack(dev(T), dev(p), dev(Y), None, X, None)
        Z = dev(Zt)
        ctx.ann_reset_optimizer()
        if sliced:
            el = np.concatenate([ctx.ann_train(X, Z, 2, batch=256, epoch0=e0, epochs_total=4)[0] for e0 in (0, 2)])
        else:
            el = ctx.ann_train(X, Z, 4, batch=256)[0]
        outs.append((ctx.ann_get_weights(), el))
    announce(f"schedule slices: epoch losses {outs[0][1]} vs {outs[1][1]}")
    assert np.array_equal(outs[0][0], outs[1][0])
    np.testing.assert_allclose(outs[0][1], outs[1][1], rtol=1e-5)
    from paper_2402_18858_amd import chemk
    for e0, tot in ((-1, 0), (3, 4), (0, 1)):     # negative start; slice past the end; total < epochs
        with pytest.raises(chemk.ChemkError):
            ctx.ann_train(X, Z, 2, batch=256, epoch0=e0, epochs_total=tot)
