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
    announce(f"forward: rel rms {rel_rms:.2e}, max abs {np.abs(g - o).max():.2e}")
    assert rel_rms < 2e-3
    assert np.abs(g - o).max() < 2e-2 * np.abs(o).max()


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
    announce(f"forward (network {dims}, {n} rows): rel rms {rel_rms:.2e}, max abs {np.abs(g - o).max():.2e}")
    assert rel_rms < 2e-3
    assert np.abs(g - o).max() < 2e-2 * np.abs(o).max()


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


def test_ann_advance_matches_oracle_post_step():
    """ANN mode of chemk_advance against the oracle: the oracle network (same
    BF16 rounding points), the oracle's post step (negative entries zeroed,
    element projection) and T from the conserved enthalpy.  Random weights
    with a 1e-3 output scale drive many species negative, so the clipping is
    exercised on most cells."""
    import oracle
    import torch
    from paper_2402_18858_amd import chemk
    mech = sm.mech_medium()
    ctx, dims, params = _ctx_small_net(mech, seed=11)
    n = 1000
    T, p, Y = _states(mech, n, 44)
    mu_x, sd_x = _set_norm(ctx, mech, T, p, Y)
    Tt, Yt = dev(T), dev(Y)
    st = torch.full((n,), -1, dtype=torch.int32, device="cuda:0")
    ctx.advance(Tt, dev(p), Yt, 5e-7, st, None, opts=chemk.default_opts(mode=chemk.MODE_ANN))
    s, Yg, Tg = host(st), host(Yt), host(Tt)
    Ws, bs = _unpack(params, dims)
    o, _ = oann.forward(Ws, bs, _oracle_inputs(T, p, Y, mu_x, sd_x), quantize=True)
    E = oann.element_matrix(mech.composition, mech.element_mass)
    assert (Y + 1e-3 * o < 0).any(1).mean() > 0.5
    Yo = oann.post_state(E, Y, 1e-3 * o)
    om = oracle.OracleMech(mech)
    _, h0 = om.thermo_batch(T, Y)
    # T: the oracle's Newton on the GPU's own Y (pure FP64, no network in it)
    To, sto = om.T_from_h_batch(h0, Yg, T)
    net = (s == 0) & (sto == 0)
    d = Yg[net] - Yo[net]
    dy = 1e-3 * o[net]
    rel_rms = np.sqrt(np.mean(d * d)) / np.sqrt(np.mean(dy * dy))
    announce(f"ann advance: {net.sum()} network cells, rel rms dY vs oracle {rel_rms:.2e}, "
             f"max |dY| {np.abs(d).max():.2e}, max |T - T(h0, Y)| "
             f"{np.abs(Tg[net] - To[net]).max():.2e} K, routed {(s != 0).sum()}")
    assert net.mean() > 0.9
    # the bar of the forward test: BF16 rounding of activations can flip
    # between FP32 (MFMA) and FP64 accumulation, one BF16 ulp at a time
    assert rel_rms < 2e-3
    assert np.abs(d).max() < 2e-2 * np.abs(dy).max()
    assert np.abs(Tg[net] - To[net]).max() < 1e-8 * T.max()
    assert Yg[net].min() >= -1e-20
    m0, m1 = element_mass(mech, Y[net]), element_mass(mech, Yg[net])
    assert (np.abs(m1 - m0) / np.maximum(m0, 1e-300))[m0 > 1e-12].max() < 1e-12


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
    hist = train.train_network(ctx, data, 1e-6, epochs=80, batch=1024, log=announce)
    assert hist["loss"][-1] < 0.5 * hist["loss"][0]
    hold = hist["holdout_index"]
    T, p, Y, Yn, _ = data
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
    train.train_network(ctx, data, 1e-6, epochs=3, batch=1024, log=announce)
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
