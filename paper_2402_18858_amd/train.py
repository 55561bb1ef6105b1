"""Training-data generation and training of the MLP that stands in for DI.

Everything numeric runs in libchemk: the DI kernel integrates the ignition
trajectories and labels every pair, the property kernels give temperatures,
and the network is fitted by the library's own forward/backward GEMM and
Adam kernels (chemk_ann_train_step).  This module only sequences the calls,
draws seeded random numbers and keeps the bookkeeping (splits, schedules).

Data recipe (paper Sec. II.B, adapted to the synthetic mechanisms):
  * 0-D constant-pressure ignition trajectories from fuel/air at
    phi ~ U[0.5, 1.5], T0 ~ U[900, 1500] K, recorded on a geometric time grid
    and perturbed by 5 % Gaussian noise on Y and 20 K on T;
  * mixing-line states between cold fuel/air (300-600 K) and burnt states
    (the paper's remedy for entrainment states, Sec. II.B);
  * states of the flame-block recipe drawn with seeds disjoint from the
    benchmark's (coverage of the LES-like cell population);
  * labels: DI over dt; 10 % of the pairs are held out and judged against DI.
"""
from __future__ import annotations

import math
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def mlp_flops_per_cell(dims):
    """Algorithmic FLOPs of one forward pass (2 per multiply-add, unpadded)."""
    return sum(2 * dims[i] * dims[i + 1] for i in range(len(dims) - 1))


def default_dims(K):
    return [K + 2, 1024, 512, 256, K]


def init_params(dims, seed):
    """He-uniform weights, zero biases, in the public parameter layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(dims) - 1):
        lim = math.sqrt(6.0 / dims[i])
        parts.append(rng.uniform(-lim, lim, dims[i] * dims[i + 1]).astype(np.float32))
        parts.append(np.zeros(dims[i + 1], np.float32))
    return np.concatenate(parts)


def species_slice(params, dims, k):
    """Public parameter vector of the one-output network of species k cut
    from a K-output network's (dims[-1] = K): every hidden layer unchanged,
    column k of the output layer's weights and its bias k."""
    off = 0
    parts = []
    L = len(dims) - 1
    for i in range(L):
        nw = dims[i] * dims[i + 1]
        W = params[off:off + nw]
        b = params[off + nw:off + nw + dims[i + 1]]
        off += nw + dims[i + 1]
        if i < L - 1:
            parts += [W, b]
        else:
            parts += [W.reshape(dims[i], dims[i + 1])[:, k].copy(), b[k:k + 1].copy()]
    assert off == params.size
    return np.concatenate(parts).astype(np.float32)


def _advance(ctx, T, P, Y, dt, st, max_steps=100000):
    from . import chemk
    ctx.advance(T, P, Y, dt, st, None, opts=chemk.default_opts(max_steps=max_steps))


def generate_pairs(ctx, mech, dt, n_pairs, seed=3001, frac_traj=0.6, frac_mix=0.1,
                   n_rec=200, t_end=2.5, log=print):
    """Returns host arrays (T, p, Y, Y_next, kind, T_next) of n_pairs DI-labelled
    pairs."""
    from synth import workload as sw

    rng = np.random.default_rng(seed)
    n_traj_states = int(n_pairs * frac_traj)
    n_mix = int(n_pairs * frac_mix)
    n_blk = n_pairs - n_traj_states - n_mix
    n_traj = max(1, int(math.ceil(n_traj_states / n_rec)))
    TT, YY, ok, p0, _, burnt_T, burnt_Y = _trajectories(ctx, mech, n_traj, n_rec, t_end, seed, log)
    sel = rng.choice(np.nonzero(ok)[0], n_traj_states, replace=n_traj_states > ok.sum())
    Tt, Yt = sw.perturb_states(TT[sel], YY[sel], seed + 2)
    # --- mixing lines: cold fuel/air <-> burnt trajectory end states ---
    j = rng.integers(0, n_traj, n_mix)
    Tc, _, Yc, _ = sw.ignition_initial_states(mech, n_mix, seed + 3, T0_range=(300.0, 600.0))
    c = rng.uniform(0.0, 1.0, n_mix)
    Tm = (1 - c) * Tc + c * burnt_T[j]
    Ym = (1 - c)[:, None] * Yc + c[:, None] * burnt_Y[j]
    # --- flame-block states with disjoint seeds ---
    Tb_l, Yb_l = [], []
    got, s_ = 0, seed + 100
    while got < n_blk:
        Tb, _, Yb, _ = sw.flame_block(mech, 32, s_)
        Tb_l.append(Tb)
        Yb_l.append(Yb)
        got += Tb.size
        s_ += 1
    Tb = np.concatenate(Tb_l)[:n_blk]
    Yb = np.concatenate(Yb_l)[:n_blk]
    Tin = np.concatenate([Tt, Tm, Tb])
    Yin = np.concatenate([Yt, Ym, Yb])
    kind = np.concatenate([np.zeros(len(Tt), np.int8), np.ones(n_mix, np.int8),
                           np.full(n_blk, 2, np.int8)])
    pin = np.full(Tin.size, p0[0])
    return _label(ctx, dt, Tin, pin, Yin, kind, log)


def _trajectories(ctx, mech, n_traj, n_rec, t_end, seed, log):
    """0-D constant-pressure ignition trajectories from fuel/air (phi ~ U[0.5,
    1.5], T0 ~ U[900, 1500] K) integrated by DI on the GPU and recorded on a
    geometric time grid.  Returns the records flattened (T, Y), a mask of the
    records of trajectories that finished, p0, phi, and the end states."""
    import torch

    from synth import workload as sw

    dev = "cuda:0"
    t0 = time.time()
    T0, p0, Y0, phi = sw.ignition_initial_states(mech, n_traj, seed + 1)
    T = torch.from_numpy(T0).to(dev)
    Y = torch.from_numpy(Y0).to(dev)
    P = torch.from_numpy(p0).to(dev)
    st = torch.zeros(n_traj, dtype=torch.int32, device=dev)
    times = np.geomspace(1e-6, t_end, n_rec)
    recT, recY = [], []
    t_prev = 0.0
    for t in times:
        _advance(ctx, T, P, Y, t - t_prev, st)
        t_prev = t
        recT.append(T.clone())
        recY.append(Y.clone())
    torch.cuda.synchronize()
    TT = torch.stack(recT, 1).reshape(-1).cpu().numpy()
    YY = torch.stack(recY, 1).reshape(-1, mech.K).cpu().numpy()
    ok = np.repeat(st.cpu().numpy() == 0, n_rec)
    log(f"train data: {n_traj} trajectories x {n_rec} records in {time.time() - t0:.1f} s")
    return TT, YY, ok, p0, phi, recT[-1].cpu().numpy(), recY[-1].cpu().numpy()


def _label(ctx, dt, Tin, pin, Yin, kind, log):
    """DI over dt on the GPU for every state; failed cells are dropped.
    Returns (T, p, Y, Y_next, kind, T_next)."""
    import torch

    dev = "cuda:0"
    t1 = time.time()
    Tg = torch.from_numpy(np.ascontiguousarray(Tin)).to(dev)
    Yg = torch.from_numpy(np.ascontiguousarray(Yin)).to(dev)
    Pg = torch.from_numpy(np.ascontiguousarray(pin)).to(dev)
    stg = torch.zeros(Tin.size, dtype=torch.int32, device=dev)
    _advance(ctx, Tg, Pg, Yg, dt, stg)
    torch.cuda.synchronize()
    good = stg.cpu().numpy() == 0
    log(f"train data: {Tin.size} DI labels in {time.time() - t1:.1f} s "
        f"({(~good).sum()} failed, dropped)")
    return (Tin[good], pin[good], np.ascontiguousarray(Yin[good]), Yg.cpu().numpy()[good],
            kind[good], Tg.cpu().numpy()[good])


# Constraint windows of the paper's recipe for methane/air (Sec. II.B): molar
# H/C and O/N of the perturbed states and their equivalence ratio.
HFRD_HC = (2.65, 4.67)
HFRD_ON = (0.254, 0.320)
HFRD_PHI = (0.20, 1.15)


def hfrd_windows(mech, phi_base):
    """The recipe's windows for this mechanism: H/C and O/N as the paper gives
    them for methane/air (the synthetic mechanisms burn CH4 in air; H/C only
    where the mechanism has carbon), and the equivalence-ratio window widened
    to the base states' range where that is wider (these trajectories reach
    phi = 1.5, richer than the paper's flames)."""
    el = list(mech.elements)
    hc = HFRD_HC if ("C" in el and "H" in el) else None
    phi = (min(HFRD_PHI[0], float(np.min(phi_base))), max(HFRD_PHI[1], float(np.max(phi_base))))
    return [hc, HFRD_ON, phi]


def generate_pairs_hfrd(ctx, mech, dt, n_pairs, seed=3001, frac_mix=0.1, frac_block=0.3, n_rec=200,
                        t_end=2.5, log=print):
    """DI-labelled pairs by the paper's hybrid flamelet/random recipe (Sec.
    II.B), with 0-D ignition trajectories standing in for the flamelet
    solutions (no 1-D flame solver here):
      * base states: the trajectory records (the same trajectories as
        generate_pairs) and, for the preheat zone of a flamelet, each
        trajectory's fresh mixture at temperatures between 300 K and its
        initial temperature (a quarter as many states as records), and
        frac_block * n_pairs flame-block states drawn with generate_pairs'
        seeds;
      * perturbed states, 1 - frac_mix of the pairs: Eqs. 3-6 with alpha =
        0.125, beta = 10, theta = 0.1, kept inside the H/C, O/N and
        equivalence-ratio windows (hfrd_windows) and 300-3000 K;
      * mixing line, frac_mix of the pairs: linear interpolation in T and Y
        between the equilibrium end states of the leanest 1 % of the
        trajectories and ambient air at 300 K (the paper's remedy for the
        lean, air-diluted states of its flames);
      * labels: DI over dt.
    Returns the same tuple as generate_pairs (kind 0 perturbed, 1 mixing line)."""
    from synth import workload as sw

    rng = np.random.default_rng(seed + 7)
    n_mix = int(n_pairs * frac_mix)
    n_pert = n_pairs - n_mix
    n_traj = max(1, int(math.ceil(0.6 * n_pairs / n_rec)))
    TT, YY, ok, p0, phi, burnt_T, burnt_Y = _trajectories(ctx, mech, n_traj, n_rec, t_end, seed, log)
    base = np.nonzero(ok)[0]
    # the preheat side of a premixed flamelet, which the ignition records lack:
    # the fresh mixture of each trajectory between 300 K and its initial T
    n_pre = n_rec // 4
    T0 = TT.reshape(n_traj, n_rec)[:, 0]
    Y0 = YY.reshape(n_traj, n_rec, -1)[:, 0]
    Tpre = 300.0 + (T0 - 300.0)[:, None] * rng.uniform(0.0, 1.0, (n_traj, n_pre))
    # flame-block states with the seeds generate_pairs uses: the synthetic
    # counterpart of the paper's flamelet solutions, which come from the same
    # flames as the states to be predicted (here the block's cold, front and
    # burnt cells and their minor-species content)
    n_blk = int(frac_block * n_pairs)
    Tb_l, Yb_l = [], []
    got, s_ = 0, seed + 100
    while got < n_blk:
        Tb, _, Yb, _ = sw.flame_block(mech, 32, s_)
        Tb_l.append(Tb)
        Yb_l.append(Yb)
        got += Tb.size
        s_ += 1
    bT = np.concatenate([TT[base], Tpre.reshape(-1)] + Tb_l)[:base.size + Tpre.size + n_blk]
    bY = np.concatenate([YY[base], np.repeat(Y0, n_pre, 0)] + Yb_l)[:bT.size]
    bP = np.full(bT.size, float(p0[0]))
    win = hfrd_windows(mech, phi)
    t0 = time.time()
    Tp, Pp, Yp, _ = sw.hfrd_states(mech, bT, bP, bY, n_pert, seed + 8, win)
    log(f"train data: {n_pert} perturbed states (windows {win}) in {time.time() - t0:.1f} s")
    lean = np.argsort(phi)[:max(1, n_traj // 100)]
    j = lean[rng.integers(0, lean.size, n_mix)]
    Ta, Pa, Ya = sw.air_states(mech, n_mix, p=float(p0[0]))
    c = rng.uniform(0.0, 1.0, n_mix)
    Tm = (1 - c) * Ta + c * burnt_T[j]
    Ym = (1 - c)[:, None] * Ya + c[:, None] * burnt_Y[j]
    Tin = np.concatenate([Tp, Tm])
    Yin = np.concatenate([Yp, Ym])
    pin = np.concatenate([Pp, Pa])
    kind = np.concatenate([np.zeros(n_pert, np.int8), np.ones(n_mix, np.int8)])
    return _label(ctx, dt, Tin, pin, Yin, kind, log)


def element_ratio_windows(mech):
    """Element-ratio windows of the input envelope, after the paper's filters on
    its training states (Sec. II.B: windows on the molar H/C and O/N ratios and
    on the equivalence ratio), as coefficients over the element mass fractions
    (a molar amount is a mass fraction over the atomic mass): H/C, O/N and the
    elemental equivalence ratio (2 n_C + n_H / 2) / n_O, each where the
    mechanism has the elements.  The bounds are placeholders until
    chemk_ann_fit_envelope fits them to the training states."""
    el = list(mech.elements)
    A = np.asarray(mech.element_mass, np.float64)

    def vec(**c):
        v = np.zeros(len(el))
        for e, x in c.items():
            if e in el:
                v[el.index(e)] = x / A[el.index(e)]
        return v

    out = []
    if "H" in el and "C" in el:
        out.append((vec(H=1.0), vec(C=1.0), 0.0, 0.0))
    if "O" in el and "N" in el:
        out.append((vec(O=1.0), vec(N=1.0), 0.0, 0.0))
    if "O" in el and ("C" in el or "H" in el):
        out.append((vec(C=2.0, H=0.5), vec(O=1.0), 0.0, 0.0))
    return out


# Defaults of the ANN path's admissibility checks (see chemk_ann_checks).
ENV_Q = 1e-3          # envelope from the 0.1 % and 99.9 % quantiles of the training states
ENV_WIDEN = 0.02      # ... widened by 2 % of that range on each side
ADJ_MAX = 3.0         # largest accepted correction, in units of the training spread of dY
NEG_TOL = 1e-6


def train_network(ctx, data, dt, epochs=50, batch=4096, lr0=1e-3, lr1=1e-5, seed=3001,
                  holdout=0.1, log=print, mech=None, adj_max=ADJ_MAX, env_q=ENV_Q, w_mass=0.0,
                  w_hrr=0.0):
    """Fits the network on the DI pairs; returns a history dict.  With `mech`
    the input envelope gets the element-ratio windows; its box, those windows
    and the dT window are fitted to the training split.  w_mass and w_hrr
    weight the mass and heat-release losses (Eqs. 9-11; chemk_ann_train_step)."""
    import torch

    dev = "cuda:0"
    T, p, Y, Yn, kind, Tn = data
    n = T.size
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    n_hold = int(n * holdout)
    hold, tr = np.sort(perm[:n_hold]), np.sort(perm[n_hold:])
    K = Y.shape[1]
    dims = default_dims(K)
    ctx.ann_create(dims)
    ctx.ann_set_weights(init_params(dims, seed))
    ctx.ann_reset_optimizer()
    Td = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in
          (("T", T[tr]), ("p", p[tr]), ("Y", Y[tr]), ("Yn", Yn[tr]))}
    ctx.ann_fit_norm(Td["T"], Td["p"], Td["Y"], Td["Yn"], dt, neg_tol=NEG_TOL)
    ctx.ann_set_checks(adj_max=adj_max, ratios=element_ratio_windows(mech) if mech is not None else ())
    Tn_tr = torch.from_numpy(np.ascontiguousarray(Tn[tr])).to(dev)
    ctx.ann_fit_envelope(Td["T"], Td["p"], Td["Y"], Tn_tr, q=env_q, widen=ENV_WIDEN)
    del Tn_tr
    ntr = tr.size
    X = torch.empty((ntr, 64), dtype=torch.int16, device=dev)
    Z = torch.empty((ntr, K), dtype=torch.float32, device=dev)
    ctx.ann_pack(Td["T"], Td["p"], Td["Y"], Td["Yn"], X, Z)
    Hd = [torch.from_numpy(np.ascontiguousarray(v[hold])).to(dev) for v in (T, p, Y, Yn)]
    Xh = torch.empty((n_hold, 64), dtype=torch.int16, device=dev)
    Zh = torch.empty((n_hold, K), dtype=torch.float32, device=dev)
    if n_hold:
        ctx.ann_pack(*Hd, Xh, Zh)
    hist = {"epochs": epochs, "batch": batch, "n_train": int(ntr), "n_holdout": int(n_hold),
            "w_mass": w_mass, "w_hrr": w_hrr}
    G = None
    if w_hrr > 0:
        G = torch.empty((ntr, K), dtype=torch.float32, device=dev)
        hist["hrr_scale"] = ctx.ann_hrr_weights(Td["T"], Td["p"], Td["Y"], Td["Yn"], dt, G)
    torch.cuda.synchronize()
    t0 = time.time()
    # the whole loop (per-epoch device-side shuffles, cosine schedule, Adam,
    # held-out loss) runs in the library: chemk_ann_train
    el, hl = ctx.ann_train(X, Z, epochs, batch=batch, lr0=lr0, lr1=lr1, seed=seed,
                           X_hold=Xh if n_hold else None, Z_hold=Zh if n_hold else None,
                           G=G, w_mass=w_mass, w_hrr=w_hrr)
    del G
    hist["loss"] = [float(v) for v in el]
    hist["hold_loss"] = [float(v) for v in hl]
    for ep in list(range(0, epochs, 10)) + [epochs - 1]:
        log(f"train: epoch {ep + 1}/{epochs} loss {el[ep]:.4e} held-out {hl[ep]:.4e}")
    step = (ntr // batch) * epochs
    hist["train_s"] = time.time() - t0
    hist["steps"] = step
    hist["holdout_index"] = hold
    return hist


def train_species_networks(ctx, data, dt, hidden=(1600, 800, 400), epochs=20, batch=4096, lr0=1e-3,
                           lr1=1e-5, seed=3001, log=print, workers=0):
    """The per-species networks of Sec. II.B: one network per mass fraction,
    hidden widths `hidden` with GELU.  Takes the normalisation, envelope and
    checks already fitted on ctx (train_network) and the same training split
    (data[-1] = the held-out indices); network k is trained as a K-output
    network whose data loss weights column k alone (a one-hot out_w), so its
    gradient flows from output k only, and keeps its hidden layers and output
    row k.  Every network starts from its own He-uniform draw and sees the
    same per-epoch row orders.

    workers = 0: all K networks train together in ctx (chemk_ann_create_species
    and chemk_ann_train: one step of all networks as grouped GEMMs), network k
    starting from the slice of its K-output draw, so that it follows the
    same steps as when trained alone.  workers >= 1: one network at a time
    as a K-output network (or that many at once, each in its own context on
    its own stream from its own host thread, the steps then without graph
    capture so that no capture is open while another thread synchronises the
    device).  Installs the K networks in ctx and returns a history dict."""
    import concurrent.futures as cf
    import threading

    import torch

    from . import chemk

    dev = "cuda:0"
    T, p, Y, Yn, hold = data
    K = Y.shape[1]
    tr = np.setdiff1d(np.arange(T.size), hold)
    norm = ctx.ann_get_norm()
    env = ctx.ann_get_envelope()
    ck = ctx.ann_get_checks()
    dims = [K + 2, *hidden, K]
    ctx.ann_create(dims)
    ctx.ann_set_norm(*norm)
    Td = [torch.from_numpy(np.ascontiguousarray(v[tr])).to(dev) for v in (T, p, Y, Yn)]
    ntr = tr.size
    X = torch.empty((ntr, 64), dtype=torch.int16, device=dev)
    Z = torch.empty((ntr, K), dtype=torch.float32, device=dev)
    ctx.ann_pack(*Td, X, Z)
    del Td
    onehot = torch.eye(K, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    dims1 = [K + 2, *hidden, 1]
    if int(workers) <= 0:
        hist = {"epochs": epochs, "batch": batch, "n_train": int(ntr), "hidden": list(hidden), "workers": 0}
        ctx.ann_create_species(dims1)
        ctx.ann_set_weights(np.concatenate([species_slice(init_params(dims, seed + 7919 * (k + 1)), dims, k)
                                            for k in range(K)]))
        ctx.ann_set_norm(*norm)
        ctx.ann_reset_optimizer()
        t0 = time.time()
        el = []
        for e0 in range(0, epochs, 5):   # slices of one schedule, to report progress
            ne = min(5, epochs - e0)
            els, _ = ctx.ann_train(X, Z, ne, batch=batch, lr0=lr0, lr1=lr1, seed=seed, epoch0=e0,
                                   epochs_total=epochs)
            el += [float(v) for v in els]
            log(f"species (grouped): epochs {e0 + 1}-{e0 + ne}/{epochs} mean loss {el[-1]:.4e} "
                f"({time.time() - t0:.0f} s)")
        torch.cuda.synchronize()
        hist["train_s"] = time.time() - t0
        hist["steps"] = (ntr // batch) * epochs * K
        hist["loss"] = el
        hist["loss_last"] = [el[-1]] * K
        ctx.ann_set_envelope(*env)
        ctx.ann_set_checks(adj_max=ck["adj_max"], dT=ck["dT"], ratios=ck["ratios"])
        return hist
    workers = max(1, min(int(workers), K))
    hist = {"epochs": epochs, "batch": batch, "n_train": int(ntr), "hidden": list(hidden),
            "workers": workers, "loss_last": [0.0] * K}
    nets = [None] * K
    lock = threading.Lock()
    t0 = time.time()

    def run(w):
        c = ctx if workers == 1 else chemk.Context(ctx.mech)
        st = None if workers == 1 else torch.cuda.Stream()
        for k in range(w, K, workers):
            c.ann_create(dims)
            c.ann_set_norm(*norm)
            c.ann_set_weights(init_params(dims, seed + 7919 * (k + 1)))
            c.ann_reset_optimizer()
            el, _ = c.ann_train(X, Z, epochs, batch=batch, lr0=lr0, lr1=lr1, seed=seed, out_w=onehot[k],
                                use_graph=workers == 1, stream=st)
            v = species_slice(c.ann_get_weights(), dims, k)
            with lock:
                nets[k] = v
                hist["loss_last"][k] = float(el[-1])
                done = sum(x is not None for x in nets)
            log(f"species {k + 1}/{K}: loss {el[0]:.3e} -> {el[-1]:.3e} ({done} done, {time.time() - t0:.0f} s)")

    if workers == 1:
        run(0)
    else:
        with cf.ThreadPoolExecutor(max_workers=workers) as ex:
            for f in [ex.submit(run, w) for w in range(workers)]:
                f.result()
    torch.cuda.synchronize()
    hist["train_s"] = time.time() - t0
    hist["steps"] = (ntr // batch) * epochs * K
    ctx.ann_create_species(dims1)
    ctx.ann_set_weights(np.concatenate(nets))
    ctx.ann_set_norm(*norm)
    ctx.ann_set_envelope(*env)
    ctx.ann_set_checks(adj_max=ck["adj_max"], dT=ck["dT"], ratios=ck["ratios"])
    return hist


def evaluate(ctx, T, p, Y, Yn_ref, hrr_scale=None):
    """Per-species RMS and max of the normalised dY error of the network
    (no projection, no fallback) against reference dY, plus the frozen-
    chemistry (dY = 0) error, on host arrays; the raw prediction's mass
    defect (mean |sum_k dY*_k|, Eq. 9) and, with the training set's
    heat-release scale, the RMS heat-release error in that unit (Eq. 10)."""
    import torch

    dev = "cuda:0"
    K = Y.shape[1]
    n = T.size
    mx, sx, my, sy, dt = ctx.ann_get_norm()
    Td = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (T, p, Y, Yn_ref)]
    X = torch.empty((n, 64), dtype=torch.int16, device=dev)
    out = torch.empty((n, K), dtype=torch.float32, device=dev)
    ctx.ann_pack(Td[0], Td[1], Td[2], None, X, None)
    ctx.ann_forward_packed(X, out)
    pred = my + sy * out.cpu().numpy().astype(np.float64)
    ref = Yn_ref - Y
    e = (pred - ref) / sy
    e0 = (0.0 - ref) / sy
    res = {"rms_norm": np.sqrt(np.mean(e * e, 0)), "max_norm": np.abs(e).max(0),
           "rms_abs": np.sqrt(np.mean((pred - ref) ** 2, 0)),
           "frozen_rms_norm": np.sqrt(np.mean(e0 * e0, 0)),
           "rms_norm_all": float(np.sqrt(np.mean(e * e))),
           "frozen_rms_norm_all": float(np.sqrt(np.mean(e0 * e0))),
           "mass_defect_mean_abs": float(np.mean(np.abs(pred.sum(1)))),
           "mass_defect_ref_mean_abs": float(np.mean(np.abs(ref.sum(1))))}
    if hrr_scale:
        G = torch.empty((n, K), dtype=torch.float32, device=dev)
        ctx.ann_hrr_weights(Td[0], Td[1], Td[2], None, dt, G, scale=hrr_scale)
        g = G.cpu().numpy().astype(np.float64)
        z = ref / sy - my / sy
        o = out.cpu().numpy().astype(np.float64)
        eh = (g * (o - z)).sum(1)
        eh0 = (g * (-my / sy - z)).sum(1)
        res.update({"hrr_rms_err": float(np.sqrt(np.mean(eh * eh))),
                    "hrr_frozen_rms_err": float(np.sqrt(np.mean(eh0 * eh0)))})
    return res


WEIGHTS = os.path.join(HERE, "weights", "mlp_medium.npz")


def weights_path(mech):
    """Stored network of a mechanism: mlp_medium.npz for the 32-species one,
    mlp_large.npz for the 53-species one."""
    name = {32: "medium", 53: "large"}.get(mech.K, f"K{mech.K}")
    return os.path.join(HERE, "weights", f"mlp_{name}.npz")


def save(ctx, path=WEIGHTS, extra=None):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    mx, sx, my, sy, dt = ctx.ann_get_norm()
    lo, hi, neg_tol = ctx.ann_get_envelope()
    ck = ctx.ann_get_checks()
    E = ctx.mech.E
    rat = ck["ratios"]
    np.savez(path, params=ctx.ann_get_weights(), dims=np.array(ctx.dims),
             species=np.array(int(getattr(ctx, "species_nets", False))), mu_x=mx, sd_x=sx,
             mu_y=my, sd_y=sy, dt=dt, env_lo=lo, env_hi=hi, neg_tol=neg_tol,
             ck_adj_max=ck["adj_max"], ck_dT=np.array(ck["dT"]),
             ck_num=np.array([r[0] for r in rat]).reshape(len(rat), E),
             ck_den=np.array([r[1] for r in rat]).reshape(len(rat), E),
             ck_lo=np.array([r[2] for r in rat]), ck_hi=np.array([r[3] for r in rat]),
             **(extra or {}))


def load(ctx, path=WEIGHTS, neg_tol=None):
    d = np.load(path, allow_pickle=False)
    dims = [int(v) for v in d["dims"]]
    if "species" in d.files and int(d["species"]):
        ctx.ann_create_species(dims)
    else:
        ctx.ann_create(dims)
    ctx.ann_set_weights(d["params"])
    ctx.ann_set_norm(d["mu_x"], d["sd_x"], d["mu_y"], d["sd_y"], float(d["dt"]))
    if "env_lo" in d.files:
        nt = float(d["neg_tol"]) if neg_tol is None else neg_tol
        ctx.ann_set_envelope(d["env_lo"], d["env_hi"], nt)
    if "ck_adj_max" in d.files:
        ctx.ann_set_checks(adj_max=float(d["ck_adj_max"]), dT=tuple(d["ck_dT"]),
                           ratios=[(d["ck_num"][j], d["ck_den"][j], d["ck_lo"][j], d["ck_hi"][j])
                                   for j in range(d["ck_lo"].size)])
    return d


def load_or_train(ctx, mech, dt, log=print, n_pairs=None, epochs=None, path=WEIGHTS):
    """Loads trained weights if present (with matching dt and dims), else runs
    the full pipeline (data generation, training) and saves the result."""
    if os.path.exists(path):
        d = np.load(path, allow_pickle=False)
        if abs(float(d["dt"]) - dt) <= 1e-12 * dt and int(d["dims"][0]) == mech.K + 2:
            load(ctx, path)
            log(f"ann: loaded {path}")
            return True
    n_pairs = n_pairs or int(os.environ.get("CHEMK_TRAIN_PAIRS", 2_000_000))
    epochs = epochs or int(os.environ.get("CHEMK_TRAIN_EPOCHS", 50))
    data = generate_pairs(ctx, mech, dt, n_pairs, log=log)
    hist = train_network(ctx, data, dt, epochs=epochs, log=log, mech=mech)
    mx, sx, my, sy, _ = ctx.ann_get_norm()
    save(ctx, path, extra={"loss": np.array(hist["loss"])})
    return True


def main(argv=None):
    """Command line: the full pipeline (DI pairs, training, held-out check),
    the weights saved to --out and a JSON report on stdout."""
    import argparse
    import json
    import sys

    import torch

    from synth import mechanism as sm

    from . import chemk

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--pairs", type=int, default=2_000_000)
    ap.add_argument("--epochs", type=int, default=50)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--dt", type=float, default=5e-7)
    ap.add_argument("--mech", default="medium", choices=["medium", "large"])
    ap.add_argument("--out", default=None)
    ap.add_argument("--w-mass", type=float, default=0.0, help="weight of the mass loss (Eq. 9)")
    ap.add_argument("--w-hrr", type=float, default=0.0, help="weight of the heat-release loss (Eq. 10)")
    ap.add_argument("--species-nets", action="store_true",
                    help="also train the per-species networks (one per mass fraction) on the same split "
                         "and report both")
    ap.add_argument("--species-hidden", default="1600,800,400")
    ap.add_argument("--species-epochs", type=int, default=20)
    ap.add_argument("--species-out", default=None, help="where to save the per-species networks")
    ap.add_argument("--species-workers", type=int, default=0,
                    help="0: all per-species networks in one grouped training; n >= 1: n of them at a "
                         "time, each as a K-output network in its own context on its own stream")
    ap.add_argument("--recipe", default="cfg4", choices=["cfg4", "hfrd"],
                    help="cfg4: noisy trajectories + mixing lines + flame-block states; "
                         "hfrd: the paper's perturbation recipe (generate_pairs_hfrd)")
    a = ap.parse_args(argv)

    def log(m):
        print(m, file=sys.stderr, flush=True)

    mech = sm.mech_medium() if a.mech == "medium" else sm.mech_large()
    a.out = a.out or weights_path(mech)
    ctx = chemk.Context(mech)
    t0 = time.time()
    gen = generate_pairs_hfrd if a.recipe == "hfrd" else generate_pairs
    data = gen(ctx, mech, a.dt, a.pairs, log=log)
    t_data = time.time() - t0
    hist = train_network(ctx, data, a.dt, epochs=a.epochs, batch=a.batch, log=log, mech=mech,
                         w_mass=a.w_mass, w_hrr=a.w_hrr)
    save(ctx, a.out, extra={"loss": np.array(hist["loss"])})
    T, p, Y, Yn = data[:4]
    hold = hist["holdout_index"]
    # the heat-release unit of the report: RMS of the label HRR over all pairs
    Tg = [torch.from_numpy(np.ascontiguousarray(v)).to("cuda:0") for v in (T, p, Y, Yn)]
    Gs = torch.empty((T.size, mech.K), dtype=torch.float32, device="cuda:0")
    hrr_unit = ctx.ann_hrr_weights(*Tg, a.dt, Gs)
    del Tg, Gs
    ev = evaluate(ctx, T[hold], p[hold], Y[hold], Yn[hold], hrr_scale=hrr_unit)
    torch.cuda.synchronize()
    fl = 3 * mlp_flops_per_cell(ctx.dims) * a.batch * hist["steps"]
    rep = {"recipe": a.recipe, "w_mass": a.w_mass, "w_hrr": a.w_hrr,
           "holdout_mass_defect": ev["mass_defect_mean_abs"],
           "holdout_mass_defect_ref": ev["mass_defect_ref_mean_abs"],
           "holdout_hrr_rms_err": ev["hrr_rms_err"], "holdout_hrr_frozen_rms_err": ev["hrr_frozen_rms_err"],
           "hrr_unit_W_m3": hrr_unit,
           "pairs": int(T.size), "n_train": hist["n_train"], "n_holdout": hist["n_holdout"],
           "epochs": a.epochs, "batch": a.batch, "data_s": t_data, "train_s": hist["train_s"],
           "train_tflops_wall": fl / hist["train_s"] / 1e12,
           "loss_first": hist["loss"][0], "loss_last": hist["loss"][-1],
           "holdout_rms_norm_all": ev["rms_norm_all"],
           "holdout_frozen_rms_norm_all": ev["frozen_rms_norm_all"],
           "holdout_rms_norm": [float(v) for v in ev["rms_norm"]],
           "holdout_max_norm": [float(v) for v in ev["max_norm"]], "weights": a.out}
    if a.species_nets:
        hidden = tuple(int(v) for v in a.species_hidden.split(","))
        hs = train_species_networks(ctx, (T, p, Y, Yn, hold), a.dt, hidden=hidden, epochs=a.species_epochs,
                                    batch=a.batch, log=log, workers=a.species_workers)
        es = evaluate(ctx, T[hold], p[hold], Y[hold], Yn[hold], hrr_scale=hrr_unit)
        torch.cuda.synchronize()
        dims1 = [mech.K + 2, *hidden, 1]
        # work done: one-output networks when grouped, K-output ones trained one by one
        fls = 3 * mlp_flops_per_cell(dims1 if hs["workers"] == 0 else dims1[:-1] + [mech.K]) * a.batch * hs["steps"]
        out_s = a.species_out or a.out.replace(".npz", "_species.npz")
        save(ctx, out_s)
        rep["species"] = {"dims": dims1, "networks": mech.K, "epochs": a.species_epochs,
                          "workers": hs["workers"],
                          "train_s": hs["train_s"], "train_tflops_wall": fls / hs["train_s"] / 1e12,
                          "loss_last": hs["loss_last"],
                          "holdout_rms_norm_all": es["rms_norm_all"],
                          "holdout_rms_norm": [float(v) for v in es["rms_norm"]],
                          "holdout_max_norm": [float(v) for v in es["max_norm"]],
                          "holdout_mass_defect": es["mass_defect_mean_abs"],
                          "holdout_hrr_rms_err": es["hrr_rms_err"], "weights": out_s}
    print(json.dumps(rep))


if __name__ == "__main__":
    main()
