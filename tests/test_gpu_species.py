"""Per-species networks (Sec. II.B: one network per mass fraction) on the GPU,
and the training features they rest on: hidden widths that are not multiples
of the 64-column slab (padded internally), per-output weights of the data
loss.  Everything against the FP64 oracle network (same BF16 rounding
points)."""
import numpy as np
import pytest

from oracle import ann as oann
from synth import mechanism as sm, workload as sw
from tests.gpu_util import announce, dev, host
from tests.test_gpu_ann import (_check_ann_step, _gpu_out, _oracle_inputs, _run_ann, _set_norm, _states,
                                _unpack)

pytestmark = pytest.mark.gpu


def _with_biases(params, dims, seed):
    rng = np.random.default_rng(seed)
    off = 0
    for i in range(len(dims) - 1):
        off += dims[i] * dims[i + 1]
        params[off:off + dims[i + 1]] = rng.normal(0, 0.1, dims[i + 1]).astype(np.float32)
        off += dims[i + 1]
    return params


def _net(mech, dims, seed):
    from paper_2402_18858_amd import chemk, train
    ctx = chemk.Context(mech)
    ctx.ann_create(dims)
    params = _with_biases(train.init_params(dims, seed), dims, seed + 1)
    ctx.ann_set_weights(params)
    return ctx, params


def _packed(ctx, T, p, Y):
    import torch
    X = torch.empty((T.size, 64), dtype=torch.int16, device="cuda:0")
    ctx.ann_pack(dev(T), dev(p), dev(Y), None, X, None)
    return X


def _grads_vs_oracle(ctx, dims, params, T, p, Y, mu_x, sd_x, Zt, out_w=None, w_mass=0.0):
    import torch
    B = T.size
    X = _packed(ctx, T, p, Y)
    idx = dev(np.arange(B, dtype=np.int32))
    grads = torch.zeros(ctx.ann_param_count(), dtype=torch.float32, device="cuda:0")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    ctx.ann_train_step(idx, X, dev(Zt), 0.0, update=False, loss=loss, grads=grads, w_mass=w_mass,
                       out_w=None if out_w is None else dev(out_w.astype(np.float32)))
    Ws, bs = _unpack(params, dims)
    o, cache = oann.forward(Ws, bs, _oracle_inputs(T, p, Y, mu_x, sd_x), quantize=True)
    K = dims[-1]
    lo, dout = oann.phys_loss(o, Zt.astype(np.float64), np.zeros(K), np.full(K, 1e-3), None, w_mass, 0.0,
                              out_w=out_w)
    gW, gb = oann.backward(Ws, bs, cache, dout, quantize=True)
    ref = np.concatenate([np.concatenate([w.ravel(), b]) for w, b in zip(gW, gb)])
    gg = host(grads).astype(np.float64)
    rel = np.sqrt(np.mean((gg - ref) ** 2)) / np.sqrt(np.mean(ref ** 2))
    return host(loss)[0], lo, rel, gg, ref


def test_hidden_widths_off_the_slab_train_like_the_oracle():
    """Hidden widths 100 and 40 (padded to 128 and 64 inside): forward and
    gradients against the oracle, then three Adam steps; the network the
    library returns then still computes what the oracle computes with the
    returned weights, so the padding units stayed at zero."""
    mech = sm.mech_medium()
    K = mech.K
    dims = [K + 2, 100, 40, K]
    ctx, params = _net(mech, dims, 31)
    T, p, Y = _states(mech, 320, 51)
    mu_x, sd_x = _set_norm(ctx, mech, T, p, Y)
    Zt = np.random.default_rng(52).normal(0, 1, (T.size, K)).astype(np.float32)
    lg, lo, rel, _, _ = _grads_vs_oracle(ctx, dims, params, T, p, Y, mu_x, sd_x, Zt)
    out = _gpu_out(ctx, T, p, Y)
    Ws, bs = _unpack(params, dims)
    o, _ = oann.forward(Ws, bs, _oracle_inputs(T, p, Y, mu_x, sd_x), quantize=True)
    f_rel = np.sqrt(np.mean((out - o) ** 2)) / np.sqrt(np.mean(o ** 2))
    announce(f"widths {dims}: forward rel rms {f_rel:.2e}; gradients rel rms {rel:.2e}; loss {lg:.6f} "
             f"(oracle {lo:.6f})")
    assert f_rel < 2e-3 and np.abs(out - o).max() < 1e-2 * o.std()
    assert rel < 1e-2 and lg == pytest.approx(lo, rel=1e-3)
    X = _packed(ctx, T, p, Y)
    idx = dev(np.arange(T.size, dtype=np.int32))
    for _ in range(3):
        ctx.ann_train_step(idx, X, dev(Zt), 1e-3, update=True)
    p3 = ctx.ann_get_weights()
    assert np.abs(p3 - params).max() > 1e-4          # the weights moved
    out3 = _gpu_out(ctx, T, p, Y)
    W3, b3 = _unpack(p3, dims)
    o3, _ = oann.forward(W3, b3, _oracle_inputs(T, p, Y, mu_x, sd_x), quantize=True)
    r3 = np.sqrt(np.mean((out3 - o3) ** 2)) / np.sqrt(np.mean(o3 ** 2))
    announce(f"after 3 Adam steps: forward rel rms {r3:.2e} against the oracle on the returned weights")
    assert r3 < 2e-3 and np.abs(out3 - o3).max() < 1e-2 * o3.std()


@pytest.mark.parametrize("kind", ["one_hot", "random"])
def test_output_weights_match_oracle(kind):
    """Per-output weights of the data loss: one-hot (the loss of one species'
    network) and random weights, with the mass term on top; loss and
    gradients against the oracle."""
    mech = sm.mech_medium()
    K = mech.K
    dims = [K + 2, 128, 64, K]
    ctx, params = _net(mech, dims, 33)
    T, p, Y = _states(mech, 256, 53)
    mu_x, sd_x = _set_norm(ctx, mech, T, p, Y)
    rng = np.random.default_rng(54)
    Zt = rng.normal(0, 1, (T.size, K)).astype(np.float32)
    if kind == "one_hot":
        w = np.zeros(K)
        w[7] = 1.0
    else:
        w = rng.uniform(0.0, 3.0, K).astype(np.float32).astype(np.float64)
    lg, lo, rel, gg, ref = _grads_vs_oracle(ctx, dims, params, T, p, Y, mu_x, sd_x, Zt, out_w=w, w_mass=0.3)
    announce(f"out_w {kind}: gradients rel rms {rel:.2e}; loss {lg:.6f} (oracle {lo:.6f})")
    assert lg == pytest.approx(lo, rel=1e-3)
    assert rel < 1e-2
    if kind == "one_hot":
        # without the mass term only column 7 of the output layer moves
        import torch
        X = _packed(ctx, T, p, Y)
        grads = torch.zeros(ctx.ann_param_count(), dtype=torch.float32, device="cuda:0")
        ctx.ann_train_step(dev(np.arange(T.size, dtype=np.int32)), X, dev(Zt), 0.0, update=False, grads=grads,
                           out_w=dev(w.astype(np.float32)))
        g = host(grads)
        nl = sum(dims[i] * dims[i + 1] + dims[i + 1] for i in range(len(dims) - 2))
        Wg = g[nl:nl + dims[-2] * K].reshape(dims[-2], K)
        bg = g[nl + dims[-2] * K:]
        others = np.arange(K) != 7
        assert np.all(Wg[:, others] == 0.0) and np.all(bg[others] == 0.0)
        assert np.abs(Wg[:, 7]).max() > 0.0
    X = _packed(ctx, T, p, Y)
    idx = dev(np.arange(T.size, dtype=np.int32))
    for bad in (np.zeros(K), np.r_[-1.0, np.ones(K - 1)], np.r_[np.nan, np.ones(K - 1)]):
        with pytest.raises(Exception):
            ctx.ann_train_step(idx, X, dev(Zt), 0.0, update=False, out_w=dev(bad.astype(np.float32)))


def _species_ctx(mech, dims1, nets_params):
    """A context holding the K one-output networks dims1 = [K+2, ..., 1]."""
    from paper_2402_18858_amd import chemk
    ctx = chemk.Context(mech)
    ctx.ann_create_species(dims1)
    ctx.ann_set_weights(np.concatenate(nets_params))
    return ctx


@pytest.mark.parametrize("hidden", [(128,), (128, 64)], ids=["one_hidden", "two_hidden"])
def test_species_networks_equal_the_k_output_network_they_are_cut_from(hidden):
    """K one-output networks cut from a K-output network (hidden layers
    shared, output column k) run as the ensemble must give the K-output
    network's outputs.  One hidden layer: the first-layer product and the
    block-diagonal output product see the same BF16 operands and FP32 sums as
    the K-output network, with only exact zeros added, so the outputs are
    bitwise equal.  Two: the output layer is fused into the grouped last
    hidden layer, whose FP32 sums run in another order (within 1e-5 of the
    outputs' spread).  Rows: several 128-row tiles and a ragged tail."""
    from paper_2402_18858_amd import train
    mech = sm.mech_medium()
    K = mech.K
    dims = [K + 2, *hidden, K]
    ctx, params = _net(mech, dims, 35)
    T, p, Y = _states(mech, 700, 55)
    mu_x, sd_x = _set_norm(ctx, mech, T, p, Y)
    out1 = _gpu_out(ctx, T, p, Y)
    ens = _species_ctx(mech, dims[:-1] + [1], [train.species_slice(params, dims, k) for k in range(K)])
    _set_norm(ens, mech, T, p, Y)
    one = dims[:-1] + [1]
    assert ens.ann_param_count() == K * sum(d * e + e for d, e in zip(one[:-1], one[1:]))
    np.testing.assert_array_equal(ens.ann_get_weights(),
                                  np.concatenate([train.species_slice(params, dims, k) for k in range(K)]))
    out2 = _gpu_out(ens, T, p, Y)
    d = np.abs(out2 - out1)
    announce(f"ensemble {hidden} vs the K-output network: max |diff| {d.max():.3e} "
             f"({(d == 0).mean() * 100:.2f} % of outputs bitwise equal), outputs' spread {out1.std():.3e}")
    if len(hidden) == 1:
        assert d.max() == 0.0
    else:
        assert d.max() <= 1e-5 * out1.std()


def test_species_networks_match_oracle_and_drive_the_advance():
    """K distinct random networks 34-96-72-1 (padded to 128 and 128 inside)
    against the oracle's per-species forward on 700 rows; the ANN step of
    chemk_advance on them against the oracle post step; the forward over more
    rows than one chunk holds (two chunks of 65,536 rows and a ragged tail),
    sampled at the chunk edges."""
    import torch
    from paper_2402_18858_amd import train
    mech = sm.mech_medium()
    K = mech.K
    dims1 = [K + 2, 96, 72, 1]
    nets = [_with_biases(train.init_params(dims1, 100 + k), dims1, 200 + k) for k in range(K)]
    ens = _species_ctx(mech, dims1, nets)
    T, p, Y = _states(mech, 700, 56)
    mu_x, sd_x = _set_norm(ens, mech, T, p, Y)
    out = _gpu_out(ens, T, p, Y)
    o = oann.species_forward([_unpack(v, dims1) for v in nets], _oracle_inputs(T, p, Y, mu_x, sd_x))
    rel = np.sqrt(np.mean((out - o) ** 2)) / np.sqrt(np.mean(o ** 2))
    announce(f"ensemble {K} x {dims1}: rel rms {rel:.2e}, max {np.abs(out - o).max():.2e} "
             f"(spread {o.std():.2e})")
    assert rel < 2e-3 and np.abs(out - o).max() < 1e-2 * o.std()
    # the ANN step on the ensemble's output
    n = 3000
    T, p, Y = _states(mech, n, 57)
    rng = np.random.default_rng(58)
    raw = oann.raw_features(T, p, Y)
    mu_x, sd_x = oann.norm_stats(raw)
    sd_y = 10.0 ** rng.uniform(-5.5, -2.5, K)
    ens.ann_set_norm(mu_x, sd_x, np.zeros(K), sd_y, 5e-7)
    ens.ann_set_checks(adj_max=2.5, dT=(-40.0, 60.0))
    Tg, Yg, sg = _run_ann(ens, T, p, Y, 5e-7)
    routed, net = _check_ann_step(mech, ens, T, p, Y, Tg, Yg, sg, ens.ann_get_checks(),
                                  f"ensemble ANN step ({n} cells)")
    assert net.sum() > 0 and routed.sum() > 0
    # 2 x 32 x (128 + 128) B of activations per row: a chunk is the 65,536-row cap
    chunk = 65536
    n = 2 * chunk + 333
    T, p, Y = _states(mech, n, 61)
    X = _packed(ens, T, p, Y)
    outd = torch.empty((n, K), dtype=torch.float32, device="cuda:0")
    ens.ann_forward_packed(X, outd)
    rows = np.unique(np.r_[np.arange(0, 32), np.arange(chunk - 32, chunk + 32),
                           np.arange(2 * chunk - 32, 2 * chunk + 32), np.arange(n - 32, n)])
    o = oann.species_forward([_unpack(v, dims1) for v in nets],
                             _oracle_inputs(T[rows], p[rows], Y[rows], mu_x, sd_x))
    g = host(outd)[rows].astype(np.float64)
    rel = np.sqrt(np.mean((g - o) ** 2)) / np.sqrt(np.mean(o ** 2))
    announce(f"ensemble forward over chunk edges ({n} rows), {rows.size} rows: rel rms {rel:.2e}")
    assert rel < 2e-3 and np.abs(g - o).max() < 1e-2 * o.std()


def test_species_networks_graph_replays_match_eager():
    """ANN mode with use_graph=1 on per-species networks: replays of the
    captured step equal the eager step bitwise (eager work in between); then
    the context switches to one K-output network and back to per-species
    networks, and each time the next captured step again equals the eager
    one (no graph of the previous network is replayed)."""
    import torch
    from paper_2402_18858_amd import chemk, train
    mech = sm.mech_medium()
    K = mech.K
    dims1 = [K + 2, 96, 72, 1]
    nets = [_with_biases(train.init_params(dims1, 600 + k), dims1, 700 + k) for k in range(K)]
    ctx = _species_ctx(mech, dims1, nets)
    n = 3000
    T, p, Y = _states(mech, n, 62)
    raw = oann.raw_features(T, p, Y)
    mu_x, sd_x = oann.norm_stats(raw)
    sd_y = 10.0 ** np.random.default_rng(63).uniform(-5.5, -2.5, K)

    def setup_norm():
        ctx.ann_set_norm(mu_x, sd_x, np.zeros(K), sd_y, 5e-7)
        ctx.ann_set_checks(adj_max=2.5, dT=(-40.0, 60.0))

    setup_norm()
    Pt, Tt, Yt = dev(p), dev(T), dev(Y)
    st = torch.full((n,), -1, dtype=torch.int32, device="cuda:0")
    og = chemk.default_opts(mode=chemk.MODE_ANN, use_graph=1)

    def graph_step():
        Tt.copy_(dev(T))
        Yt.copy_(dev(Y))
        st.fill_(-1)
        ctx.advance(Tt, Pt, Yt, 5e-7, st, None, opts=og)
        torch.cuda.synchronize()
        return host(Tt), host(Yt), host(st)

    outs = []
    for phase in range(3):
        ref = _run_ann(ctx, T, p, Y, 5e-7)
        for rep in range(3):
            got = graph_step()
            for a_, b_ in zip(ref, got):
                assert np.array_equal(a_, b_), (phase, rep)
            _run_ann(ctx, T[:300], p[:300], Y[:300], 5e-7)
        nr = int(((ref[2] & chemk.CELL_ROUTED_DI) != 0).sum())
        announce(f"species graph phase {phase}: 3 replays equal the eager step ({nr} routed)")
        outs.append(ref[1])
        if phase == 0:
            dims = [K + 2, 128, 64, K]
            ctx.ann_create(dims)
            ctx.ann_set_weights(_with_biases(train.init_params(dims, 64), dims, 65))
            setup_norm()
        elif phase == 1:
            ctx.ann_create_species(dims1)
            ctx.ann_set_weights(np.concatenate(nets))
            setup_norm()
    # back on the same networks: the same result as the first phase
    assert np.array_equal(outs[0], outs[2])
    assert not np.array_equal(outs[0], outs[1])


def test_species_networks_at_paper_size_on_the_flame_block():
    """The paper's per-species networks (hidden 1600-800-400, GELU) for all
    K = 32 species, random weights, on the 262,144-cell flame block in the
    launch configuration of the timed ensemble forward (chunks of 17,408
    rows): sampled rows (chunk edges and random ones) against the oracle."""
    import torch
    from paper_2402_18858_amd import train
    mech = sm.mech_medium()
    K = mech.K
    dims1 = [K + 2, 1600, 800, 400, 1]
    nets = [_with_biases(train.init_params(dims1, 300 + k), dims1, 400 + k) for k in range(K)]
    ens = _species_ctx(mech, dims1, nets)
    T, p, Y, _ = sw.flame_block(mech, 64, 2002)
    mu_x, sd_x = oann.norm_stats(oann.raw_features(T[::64], p[::64], Y[::64]))
    ens.ann_set_norm(mu_x, sd_x, np.zeros(K), np.full(K, 1e-3), 5e-7)
    n = T.size
    X = _packed(ens, T, p, Y)
    out = torch.empty((n, K), dtype=torch.float32, device="cuda:0")
    ens.ann_forward_packed(X, out)
    g_all = host(out)
    rng = np.random.default_rng(59)
    ch = 17408
    rows = np.unique(np.r_[np.arange(0, 16), np.arange(ch - 16, ch + 16), np.arange(15 * ch - 16, 15 * ch + 16),
                           np.arange(n - 16, n), rng.choice(n, 64, replace=False)])
    o = oann.species_forward([_unpack(v, dims1) for v in nets],
                             _oracle_inputs(T[rows], p[rows], Y[rows], mu_x, sd_x))
    g = g_all[rows].astype(np.float64)
    rel = np.sqrt(np.mean((g - o) ** 2)) / np.sqrt(np.mean(o ** 2))
    announce(f"paper-size ensemble on {n} cells, {rows.size} sampled rows: rel rms {rel:.2e}, max "
             f"{np.abs(g - o).max():.2e} (spread {o.std():.2e})")
    assert np.isfinite(g_all).all()
    assert rel < 2e-3 and np.abs(g - o).max() < 2e-2 * o.std()


def test_species_networks_one_hidden_layer_train_and_refuse_physics_losses():
    """Per-species networks with one hidden layer (the first layer dense, the
    output layer block diagonal, no grouped layer) train: the loss of a
    step matches the oracle's and falls over a few steps.  The physics
    losses and per-output weights, which couple species, are refused; so are
    shapes that are not one-output networks."""
    import torch
    from paper_2402_18858_amd import chemk, train
    mech = sm.mech_medium()
    K = mech.K
    dims1 = [K + 2, 64, 1]
    nets = [train.init_params(dims1, k) for k in range(K)]
    ens = _species_ctx(mech, dims1, nets)
    B = 128
    T, p, Y = _states(mech, B, 60)
    mu_x, sd_x = _set_norm(ens, mech, T, p, Y)
    X = _packed(ens, T, p, Y)
    Zh = np.random.default_rng(61).normal(0, 1, (B, K)).astype(np.float32)
    Zt = dev(Zh)
    idx = dev(np.arange(B, dtype=np.int32))
    loss = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    ens.ann_train_step(idx, X, Zt, 0.0, update=False, loss=loss)
    xin = _oracle_inputs(T, p, Y, mu_x, sd_x)
    lo = np.mean([oann.mse_loss(oann.forward(*_unpack(nets[k], dims1), xin, quantize=True)[0],
                                Zh[:, k:k + 1].astype(np.float64))[0] for k in range(K)])
    l0 = host(loss)[0]
    assert l0 == pytest.approx(lo, rel=1e-3)
    for _ in range(20):
        ens.ann_train_step(idx, X, Zt, 3e-3, update=True)
    loss.zero_()
    ens.ann_train_step(idx, X, Zt, 0.0, update=False, loss=loss)
    announce(f"one hidden layer, grouped steps: loss {l0:.4f} (oracle {lo:.4f}) -> {host(loss)[0]:.4f} after 20")
    assert host(loss)[0] < 0.9 * l0
    for kw in ({"w_mass": 0.5}, {"out_w": dev(np.ones(K, np.float32))}):
        with pytest.raises(chemk.ChemkError):
            ens.ann_train_step(idx, X, Zt, 1e-3, **kw)
    with pytest.raises(chemk.ChemkError):
        ens.ann_train(X, Zt, 1, batch=128, w_mass=0.5)
    ctx = chemk.Context(mech)
    for bad in ([K + 2, 1], [K + 2, 64, 2], [K + 1, 64, 1]):
        with pytest.raises(chemk.ChemkError):
            ctx.ann_create_species(bad)


def test_species_training_on_four_streams_equals_one_at_a_time():
    """train_species_networks with four networks training at once (own
    contexts, streams and host threads, eager steps) gives every network
    bitwise the weights of the one-at-a-time run (graph-replayed steps): the
    steps are deterministic and the networks independent."""
    import torch
    from paper_2402_18858_amd import chemk, train
    mech = sm.mech_medium()
    K = mech.K
    n = 4096 + 512
    T, p, Y = _states(mech, n, 66)
    rng = np.random.default_rng(67)
    Yn = np.clip(Y + rng.normal(0, 1e-4, Y.shape) * Y, 0.0, None)
    Yn /= Yn.sum(1, keepdims=True)
    hold = np.arange(n - 512, n)
    outs = []
    for workers in (1, 4):
        ctx = chemk.Context(mech)
        ctx.ann_create([K + 2, 64, K])
        # the same normalisation for both runs, from the host (the device fit
        # sums with atomics, in no fixed order)
        mu_x, sd_x = oann.norm_stats(oann.raw_features(T[:n - 512], p[:n - 512], Y[:n - 512]))
        d = (Yn - Y)[:n - 512]
        ctx.ann_set_norm(mu_x, sd_x, d.mean(0), np.maximum(d.std(0), 1e-12), 5e-7)
        h = train.train_species_networks(ctx, (T, p, Y, Yn, hold), 5e-7, hidden=(96, 40), epochs=2, batch=1024,
                                         log=lambda m: None, workers=workers)
        torch.cuda.synchronize()
        outs.append(ctx.ann_get_weights())
        announce(f"species training, {workers} worker(s): {h['train_s']:.2f} s, last losses "
                 f"{min(h['loss_last']):.3e} .. {max(h['loss_last']):.3e}")
    assert np.array_equal(outs[0], outs[1])


def test_grouped_training_step_matches_oracle():
    """One training step of 32 per-species networks 34-96-72-1 trained
    together (grouped GEMMs): the batch loss (the mean of the networks' own
    losses) and every network's gradient (its output column's mean squared
    error alone) against the oracle network by network; then three Adam
    steps, after which the networks still compute what the oracle computes
    with the returned weights (the padding units stayed at zero)."""
    import torch
    from paper_2402_18858_amd import train
    mech = sm.mech_medium()
    K = mech.K
    dims1 = [K + 2, 96, 72, 1]
    nets = [_with_biases(train.init_params(dims1, 800 + k), dims1, 900 + k) for k in range(K)]
    ens = _species_ctx(mech, dims1, nets)
    B = 256
    T, p, Y = _states(mech, B, 68)
    mu_x, sd_x = _set_norm(ens, mech, T, p, Y)
    Zt = np.random.default_rng(69).normal(0, 1, (B, K)).astype(np.float32)
    X = _packed(ens, T, p, Y)
    idx = dev(np.arange(B, dtype=np.int32))
    grads = torch.zeros(ens.ann_param_count(), dtype=torch.float32, device="cuda:0")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    ens.ann_reset_optimizer()
    ens.ann_train_step(idx, X, dev(Zt), 0.0, update=False, loss=loss, grads=grads)
    gg = host(grads).astype(np.float64)
    xin = _oracle_inputs(T, p, Y, mu_x, sd_x)
    n1 = nets[0].size
    los, rels = [], []
    for k in range(K):
        Ws, bs = _unpack(nets[k], dims1)
        o, cache = oann.forward(Ws, bs, xin, quantize=True)
        lo, dout = oann.mse_loss(o, Zt[:, k:k + 1].astype(np.float64))
        gW, gb = oann.backward(Ws, bs, cache, dout, quantize=True)
        ref = np.concatenate([np.concatenate([w.ravel(), b]) for w, b in zip(gW, gb)])
        seg = gg[k * n1:(k + 1) * n1]
        los.append(lo)
        rels.append(np.sqrt(np.mean((seg - ref) ** 2)) / np.sqrt(np.mean(ref ** 2)))
    announce(f"grouped training step, {K} networks {dims1}: loss {host(loss)[0]:.6f} (oracle mean "
             f"{np.mean(los):.6f}), gradient rel rms max {max(rels):.2e}")
    assert host(loss)[0] == pytest.approx(np.mean(los), rel=1e-3)
    assert max(rels) < 1e-2
    for _ in range(3):
        ens.ann_train_step(idx, X, dev(Zt), 1e-3, update=True)
    p3 = ens.ann_get_weights()
    assert np.abs(p3 - np.concatenate(nets)).max() > 1e-4
    out3 = _gpu_out(ens, T, p, Y)
    o3 = oann.species_forward([_unpack(p3[k * n1:(k + 1) * n1], dims1) for k in range(K)], xin)
    r3 = np.sqrt(np.mean((out3 - o3) ** 2)) / np.sqrt(np.mean(o3 ** 2))
    announce(f"after 3 grouped Adam steps: forward rel rms {r3:.2e} against the oracle on the returned weights")
    assert r3 < 2e-3 and np.abs(out3 - o3).max() < 1e-2 * o3.std()


def test_grouped_training_follows_one_network_at_a_time():
    """The grouped training of all per-species networks and the one-at-a-time
    training (K-output networks with a one-hot loss weight, sliced) start
    from the same weights and see the same rows: after two epochs their
    networks agree to the rounding of the different summation orders."""
    import torch
    from paper_2402_18858_amd import chemk, train
    mech = sm.mech_medium()
    K = mech.K
    n = 4096 + 512
    T, p, Y = _states(mech, n, 70)
    rng = np.random.default_rng(71)
    Yn = np.clip(Y + rng.normal(0, 1e-4, Y.shape) * Y, 0.0, None)
    Yn /= Yn.sum(1, keepdims=True)
    hold = np.arange(n - 512, n)
    outs = []
    for workers in (0, 1):
        ctx = chemk.Context(mech)
        ctx.ann_create([K + 2, 64, K])
        mu_x, sd_x = oann.norm_stats(oann.raw_features(T[:n - 512], p[:n - 512], Y[:n - 512]))
        d = (Yn - Y)[:n - 512]
        ctx.ann_set_norm(mu_x, sd_x, d.mean(0), np.maximum(d.std(0), 1e-12), 5e-7)
        h = train.train_species_networks(ctx, (T, p, Y, Yn, hold), 5e-7, hidden=(96, 40), epochs=2, batch=1024,
                                         log=lambda m: None, workers=workers)
        torch.cuda.synchronize()
        outs.append((ctx.ann_get_weights(), _gpu_out(ctx, T[hold], p[hold], Y[hold])))
        announce(f"species training, workers={workers}: {h['train_s']:.2f} s")
    dw = np.abs(outs[0][0] - outs[1][0]).max()
    do = np.abs(outs[0][1] - outs[1][1]).max()
    announce(f"grouped vs one at a time: max |dw| {dw:.2e}, max |d out| {do:.2e} (spread {outs[1][1].std():.2e})")
    assert dw < 1e-3
    assert do < 1e-2 * outs[1][1].std()


def test_species_networks_for_53_species():
    """Per-species networks on the 53-species mechanism: 53 groups (not a
    multiple of 8) and an output count that is not a multiple of 8 (the
    block-diagonal and column-sum kernels take their element-wise paths);
    forward and one grouped training step against the oracle."""
    import torch
    from paper_2402_18858_amd import train
    mech = sm.mech_large()
    K = mech.K
    dims1 = [K + 2, 64, 40, 1]
    nets = [_with_biases(train.init_params(dims1, 1000 + k), dims1, 1100 + k) for k in range(K)]
    ens = _species_ctx(mech, dims1, nets)
    B = 192
    T, p, Y = _states(mech, B, 72)
    mu_x, sd_x = _set_norm(ens, mech, T, p, Y)
    xin = _oracle_inputs(T, p, Y, mu_x, sd_x)
    out = _gpu_out(ens, T, p, Y)
    o = oann.species_forward([_unpack(v, dims1) for v in nets], xin)
    rel = np.sqrt(np.mean((out - o) ** 2)) / np.sqrt(np.mean(o ** 2))
    Zt = np.random.default_rng(73).normal(0, 1, (B, K)).astype(np.float32)
    X = _packed(ens, T, p, Y)
    grads = torch.zeros(ens.ann_param_count(), dtype=torch.float32, device="cuda:0")
    ens.ann_train_step(dev(np.arange(B, dtype=np.int32)), X, dev(Zt), 0.0, update=False, grads=grads)
    gg = host(grads).astype(np.float64)
    n1 = nets[0].size
    rels = []
    for k in range(K):
        Ws, bs = _unpack(nets[k], dims1)
        ok, cache = oann.forward(Ws, bs, xin, quantize=True)
        _, dout = oann.mse_loss(ok, Zt[:, k:k + 1].astype(np.float64))
        gW, gb = oann.backward(Ws, bs, cache, dout, quantize=True)
        ref = np.concatenate([np.concatenate([w.ravel(), b]) for w, b in zip(gW, gb)])
        rels.append(np.sqrt(np.mean((gg[k * n1:(k + 1) * n1] - ref) ** 2)) / np.sqrt(np.mean(ref ** 2)))
    announce(f"53 per-species networks {dims1}: forward rel rms {rel:.2e}; gradient rel rms max {max(rels):.2e}")
    assert rel < 2e-3 and np.abs(out - o).max() < 1e-2 * o.std()
    assert max(rels) < 1e-2
