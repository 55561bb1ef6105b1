"""Benchmark of the per-cell chemistry advance on one MI355X.

Workload: the 64^3 block (262,144 cells) of the 32-species / 160-reaction
synthetic mechanism, stratified into cold reactants, flame-front and
product cells, advanced over dt = 5e-7 s.  A step is one chemistry advance
of the whole block: the ANN path (ingest, BF16 MLP on MFMA, FP64 element
correction and checks, DI on the routed cells) when a trained network is
available, else the DI path (stiffness binning and the persistent Rosenbrock
kernel).  Both paths are timed; `value` is the headline path's
cell-updates/s.

Timing: every timed step advances its own copy of the block's initial
state, made before the timed region; each step replays a hipGraph captured
in the untimed warm-up.  Accuracy is measured on a step from the initial
state: the ANN step against the FP64 DI step on every cell, the DI step
against the oracle (reference tolerance) on a stratified sample.  The split
of each path into phases and GEMM layers comes from separate eager steps
with HIP events around each phase's launches.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode auto|di|ann]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6       # MI355X FP64 vector
PEAK_BF16_TFLOPS = 2500.0     # MI355X dense BF16 MFMA
PEAK_HBM_GBS = 8000.0
# an FP64 exp as compiled for gfx950 (a kernel of one exp(): 19 FP64
# instructions, 13 of them FMAs) counted as 32 operations
EXP_FLOPS = 32


def di_flops_per_step(K, R):
    """Algorithmic FLOPs of one RODAS step on one cell, N = K + 1 unknowns:
    6 right-hand sides (each R reactions at 12 operations and two exp,
    plus 20 per species), one analytic Jacobian (40 per reaction, 20 per
    species), one LU of the N x N iteration matrix (2N^3/3) and 6 triangular
    solves (2N^2 each)."""
    N = K + 1
    rhs = R * (12 + 2 * EXP_FLOPS) + 20 * K
    jac = 40 * R + 20 * K
    return 6 * rhs + jac + 2.0 * N ** 3 / 3.0 + 6 * 2.0 * N * N


def measured_traffic(key, routed=None):
    """HBM bytes per launch of a kernel from the rocprofv3 FETCH_SIZE / WRITE_SIZE
    runs summarised in profiles/traffic.json (scaled by the copy calibration),
    or None when the kernel's sources changed since those counters were taken
    (or, for the routed DI launch, when this run routes another number of cells)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    entry = json.load(open(path)).get(key)
    if not entry:
        return None
    if routed is not None and entry.get("routed_cells") != routed:
        return None
    srcs = {"di_kernel": ("di.hip", "chemk_dev.h"), "di_kernel_routed": ("di.hip", "chemk_dev.h"),
            "gemm_layer2": ("gemm.hip",), "post_kernel": ("ann.hip",),
            "ingest_kernel": ("ann.hip",), "species_layer2": ("gemm.hip",)}[key]
    h = hashlib.sha1()
    for f in srcs:
        with open(os.path.join(ROOT, "paper_2402_18858_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return entry["bytes"] if h.hexdigest()[:16] == entry["sources_sha1"] else None


def closure_timing(ctx, mech, Tin, P, Yin, T_a, Y_a, dt, log, reps=10):
    """The steps either side of the advance on the block: mixture viscosity
    and conductivity (chemk_transport) and the PaSR closure of the ANN step's
    result (chemk_pasr), HIP-event timed over `reps` launches each, with their
    algorithmic HBM bytes per cell (inputs read once, outputs written once)."""
    import torch
    from synth import transport as st

    dev = "cuda:0"
    n, K = Yin.shape
    mu_c, lam_c = st.transport_fits(mech)
    ctx.transport_set(mu_c, lam_c)
    mu = torch.empty(n, dtype=torch.float64, device=dev)
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    Y1 = torch.from_numpy(np.ascontiguousarray(Y_a)).to(dev)
    rng = np.random.default_rng(9)
    ksgs = torch.from_numpy(10.0 ** rng.uniform(-1, 2, n)).to(dev)
    delta = torch.full((n,), 1e-3, dtype=torch.float64, device=dev)
    kap = torch.empty(n, dtype=torch.float64, device=dev)
    om = torch.empty((n, K), dtype=torch.float64, device=dev)
    Yb = torch.empty((n, K), dtype=torch.float64, device=dev)

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_tr = timed(lambda: ctx.transport(Tin, Yin, mu, lam))
    t_pa = timed(lambda: ctx.pasr(Tin, P, Yin, Y1, dt, ksgs, delta, mu, kappa=kap, omega=om, Y_out=Yb))
    b_tr = 8 * (1 + K) + 16                   # T, Y in; mu, lambda out
    b_pa = 8 * (2 + 2 * K + 3) + 8 * (1 + 2 * K)   # T, p, Y0, Y1, k, delta, mu in; kappa, omega, Y out
    # transport's algorithmic FP64 work: 7 operations per species pair in
    # Wilke's sum (ratio, fused multiply-add, square, product, accumulate)
    # and per species two polynomial exps (6 + EXP_FLOPS each) and about 14
    # more (mole fraction, square root, the three mixture sums)
    f_tr = 7 * K * K + (2 * (6 + EXP_FLOPS) + 14) * K
    tr_tf = f_tr * n / (t_tr * 1e-3) / 1e12
    pa_gbs = b_pa * n / (t_pa * 1e-3) / 1e9
    k_h = kap.cpu().numpy()
    log(f"closure: transport {t_tr:.3f} ms ({tr_tf:.2f} TFLOP/s), PaSR {t_pa:.3f} ms ({pa_gbs:.0f} GB/s) on {n} cells")
    return {"cells": n, "transport_ms": t_tr, "transport_bytes_per_cell": b_tr,
            "transport_GB_per_s": b_tr * n / (t_tr * 1e-3) / 1e9,
            "pasr_ms": t_pa, "pasr_bytes_per_cell": b_pa,
            "pasr_GB_per_s": pa_gbs, "peak_GB_per_s": PEAK_HBM_GBS,
            "transport_roofline": {"bound": "alu", "achieved": tr_tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                   "frac": tr_tf / PEAK_FP64_TFLOPS, "flops_per_cell": f_tr},
            "pasr_roofline": {"bound": "hbm", "achieved": pa_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                              "frac": pa_gbs / PEAK_HBM_GBS},
            "kappa_p10_p50_p90": [float(np.percentile(k_h, q)) for q in (10, 50, 90)],
            "inputs": "transport fits of synth/transport.py; k_sgs ~ 10^U[-1,2] m^2/s^2, delta = 1 mm"}


def species_timing(ctx, mech, Tin, P, Yin, log, reps=5, hidden=(1600, 800, 400)):
    """Forward of the per-species networks at the paper's size (one network
    per species, hidden 1600-800-400, GELU; random He-uniform weights, seeded)
    on the block's cells, HIP-event timed over `reps` passes on the stream the
    kernels run on; algorithmic FLOPs 2 x (multiply-adds of the unpadded
    layers) per cell and network.  Inference only: the weights play no part in
    the time."""
    import torch
    from paper_2402_18858_amd import chemk, train

    n, K = Yin.shape
    dims1 = [K + 2, *hidden, 1]
    ens = chemk.Context(mech)
    ens.ann_create_species(dims1)
    ens.ann_set_weights(np.concatenate([train.init_params(dims1, 500 + k) for k in range(K)]))
    ens.ann_set_norm(*ctx.ann_get_norm())
    X = torch.empty((n, 64), dtype=torch.int16, device="cuda:0")
    ens.ann_pack(Tin, P, Yin, None, X, None)
    out = torch.empty((n, K), dtype=torch.float32, device="cuda:0")
    ens.ann_forward_packed(X, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ens.ann_forward_packed(X, out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    fl = K * train.mlp_flops_per_cell(dims1)
    tf = fl * n / (ms * 1e-3) / 1e12
    # per layer: one more forward with the library's phase events around each
    # launch (the output layer is fused into the last hidden layer's launch;
    # its sum kernel is counted under the last layer phase)
    ens.timing(True)
    ens.ann_forward_packed(X, out)
    ph = ens.timing_read()
    ens.timing(False)
    nl = len(dims1) - 1
    lay_fl = [2 * K * dims1[i] * dims1[i + 1] for i in range(nl)]
    lay_fl[nl - 2] += lay_fl[nl - 1]
    per_layer = {}
    for i in range(min(nl - 1, 4)):
        t_ms, cnt = ph[f"layer{i + 1}"]
        if cnt == 0:
            continue
        avg = t_ms / cnt
        rows = n / cnt
        per_layer[f"layer{i + 1}"] = {"launches": cnt, "avg_launch_us": 1e3 * avg, "rows_per_launch": rows,
                                      "flops_per_launch": lay_fl[i] * rows,
                                      "tflops": lay_fl[i] * rows / (avg * 1e-3) / 1e12,
                                      "frac": lay_fl[i] * rows / (avg * 1e-3) / 1e12 / PEAK_BF16_TFLOPS}
    del ens
    if not per_layer:
        raise RuntimeError("the library recorded no layer phases for chemk_ann_forward_packed")
    dom = max(per_layer, key=lambda k_: lay_fl[int(k_[-1]) - 1])
    log(f"per-species networks {K} x {dims1}: {ms:.3f} ms per forward of {n} cells, {tf:.1f} TFLOP/s; "
        f"{dom} {per_layer[dom]['tflops']:.0f} TFLOP/s")
    return {"networks": K, "dims": dims1, "cells": n, "ms_per_forward": ms, "cells_per_s": n / (ms * 1e-3),
            "flops_per_cell": fl, "tflops": tf, "peak_tflops": PEAK_BF16_TFLOPS,
            "frac": tf / PEAK_BF16_TFLOPS, "per_layer": per_layer,
            "roofline": {"bound": "mfma", "achieved": per_layer[dom]["tflops"], "peak": PEAK_BF16_TFLOPS,
                         "unit": "TFLOP/s", "frac": per_layer[dom]["frac"],
                         # HBM bytes of a full-chunk (17,408-row) layer-2 launch, scaled to
                         # the average launch's rows like "achieved"
                         "traffic": (measured_traffic("species_layer2") * per_layer[dom]["rows_per_launch"] / 17408
                                     if dom == "layer2" and measured_traffic("species_layer2") else None),
                         "kernel": f"gemm_dma_kernel grouped over {K} networks, {dom} "
                                   f"({dims1[int(dom[-1]) - 1]} -> {dims1[int(dom[-1])]})",
                         "flops_per_launch": per_layer[dom]["flops_per_launch"]},
            "weights": "random He-uniform, seeded (the forward's time does not depend on them)"}


def element_mass(mech, Y):
    comp = mech.composition.astype(np.float64)
    Em = comp * mech.element_mass[None, :] / (comp @ mech.element_mass)[:, None]
    return Y @ Em


def ann_vs_di(mech, sd_y, Y0, T_a, Y_a, st_a, T_d, Y_d, routed_bit):
    """Error of the ANN step (network cells and routed cells together, as the
    solver sees them) against the FP64 DI step of the same cells: per-species
    RMS and max of (Y_ann - Y_di) / sd(dY), the same over the network's cells
    alone, |dT|, the routed fraction and the element-mass drift."""
    routed = (st_a & routed_bit) != 0
    net = ~routed
    e = (Y_a - Y_d) / sd_y[None, :]
    en = e[net]
    m0, m1 = element_mass(mech, Y0), element_mass(mech, Y_a)
    drift = np.abs(m1 - m0) / np.maximum(m0, 1e-300)
    dT = T_a - T_d
    return {"cells": int(Y0.shape[0]), "routed_cells": int(routed.sum()),
            "routed_fraction": float(routed.mean()),
            "rms_norm_all_species": float(np.sqrt(np.mean(e * e))),
            "max_norm_all_species": float(np.abs(e).max()),
            "rms_norm": [round(float(v), 5) for v in np.sqrt(np.mean(e * e, 0))],
            "max_norm": [round(float(v), 4) for v in np.abs(e).max(0)],
            "network_cells_rms_norm": ([round(float(v), 5) for v in np.sqrt(np.mean(en * en, 0))]
                                       if en.size else None),
            "network_cells_max_norm": [round(float(v), 4) for v in np.abs(en).max(0)] if en.size else None,
            "rms_abs": [float(f"{v:.3e}") for v in np.sqrt(np.mean((Y_a - Y_d) ** 2, 0))],
            "sd_dY_train": [float(f"{v:.3e}") for v in sd_y],
            "max_abs_T_K": float(np.abs(dT).max()),
            "rms_abs_T_K": float(np.sqrt(np.mean(dT ** 2))),
            "network_cells_max_abs_T_K": float(np.abs(dT[net]).max()) if net.any() else 0.0,
            "element_drift_max": float(drift[m0 > 1e-12].max())}


def envelope_sweep(ctx, mech, dt, Tin, P, Yin, opts, region, T_di, Y_di, sd_y, di_idx, log,
                   qs=(0.0, 1e-5, 1e-4, 3e-4, 1e-3)):
    """The envelope's quantile q against routed cells, step time and error: the
    training pairs are regenerated (same seed and split as the stored
    network's), the box, ratio windows and dT window refitted for each q, and
    one eager step of the block timed by phase; the stored envelope is
    restored at the end."""
    import torch
    from paper_2402_18858_amd import chemk, train
    data = train.generate_pairs(ctx, mech, dt, 2_000_000, log=log)
    T, p, Y, _, _, Tn = data
    perm = np.random.default_rng(3001).permutation(T.size)
    tr = np.sort(perm[int(T.size * 0.1):])
    dev = Tin.device
    Tt, Pt, Yt, Tnt = (torch.from_numpy(np.ascontiguousarray(a[tr])).to(dev) for a in (T, p, Y, Tn))
    lo0, hi0, nt0 = ctx.ann_get_envelope()
    ck0 = ctx.ann_get_checks()
    n = Tin.numel()
    st = torch.zeros(n, dtype=torch.int32, device=dev)
    out = []
    for q in qs:
        ctx.ann_set_checks(adj_max=ck0["adj_max"], dT=ck0["dT"], ratios=ck0["ratios"])
        ctx.ann_fit_envelope(Tt, Pt, Yt, Tnt, q=q, widen=train.ENV_WIDEN)
        Ta, Ya = Tin.clone(), Yin.clone()
        ctx.timing(True)
        ctx.advance(Ta, P, Ya, dt, st, None, opts=opts)
        ph = ctx.timing_read()
        ctx.timing(False)
        s_ = st.cpu().numpy()[di_idx]
        r = (s_ & chemk.CELL_ROUTED_DI) != 0
        e = (Ya.cpu().numpy()[di_idx] - Y_di) / sd_y
        eT = Ta.cpu().numpy()[di_idx] - T_di
        out.append({"q": q, "routed": int(r.sum()),
                    "routed_by_region": np.bincount(region[di_idx][r], minlength=3).tolist(),
                    "step_ms": sum(ph[k][0] for k in ("ingest", "mlp", "post", "fallback")),
                    "fallback_ms": ph["fallback"][0], "rms_norm": float(np.sqrt(np.mean(e * e))),
                    "max_norm": float(np.abs(e).max()), "T_rms_K": float(np.sqrt(np.mean(eT ** 2))),
                    "T_max_K": float(np.abs(eT).max())})
        log(f"envelope q={q:g}: {out[-1]}")
    ctx.ann_set_envelope(lo0, hi0, nt0)
    ctx.ann_set_checks(adj_max=ck0["adj_max"], dT=ck0["dT"], ratios=ck0["ratios"])
    return out


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                return ln.split(":", 1)[1].strip()
    except Exception:  # noqa: BLE001 - informational
        pass
    return "unknown"


WORKLOADS = {
    # the metric's configuration: 64^3 flame block, 32 species / 160 reactions
    "medium": dict(mech="mech_medium", nx=64, seed=2002, di_cells=None, rtol=1e-7),
    # the full step at scale: 128^3 block, 53 species / 325 reactions; DI is
    # timed and used as the accuracy reference on a stratified sample; this
    # mechanism needs rtol 5e-8 for the 1e-6 parity bar
    "large": dict(mech="mech_large", nx=128, seed=2005, di_cells=65536, rtol=5e-8),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--di-steps", type=int, default=2, help="timed DI steps (about 3 s each)")
    ap.add_argument("--mode", default="auto", choices=["auto", "di", "ann"])
    ap.add_argument("--workload", default="medium", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2400,
                    help="cells of the oracle at the GPU tolerance (about 10 s on 16 host threads)")
    ap.add_argument("--cpu-sample-ref", type=int, default=240,
                    help="cells of the oracle at the reference tolerance (rtol 1e-10)")
    ap.add_argument("--envelope-sweep", action="store_true",
                    help="also refit the envelope for several quantiles q on regenerated training "
                         "data and report routed cells, step time and error for each")
    ap.add_argument("--weights", default=None,
                    help="network weights to load (train.py --out); default: the workload's stock file")
    ap.add_argument("--di-kernel", type=int, default=0, choices=[0, 1, 2],
                    help="DI factorisation: 0 automatic, 1 LDS LU, 2 register LU")
    ap.add_argument("--no-species", action="store_true",
                    help="skip the timing of the per-species networks' forward")
    ap.add_argument("--species-only", action="store_true",
                    help="time only the per-species networks' forward on the block and print that "
                         "(not the headline metric)")
    ap.add_argument("--bins", type=int, default=0, help="fixed stiffness bins (skips the autotuner)")
    ap.add_argument("--wpc", type=int, default=0, help="fixed DI waves per CU (with --bins)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only. The chemistry advance has no cross-GPU step: "
              "cells are independent, so each further GPU would advance its own share of them.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2402_18858_amd import chemk
    from synth import mechanism as sm, workload as sw

    def log(m):
        print(f"bench.py: {m}", file=sys.stderr, flush=True)

    wl = WORKLOADS[args.workload]
    mech = getattr(sm, wl["mech"])()
    T0, p0, Y0, region = sw.flame_block(mech, wl["nx"], wl["seed"])
    n, K = Y0.shape
    dt = 5e-7
    dev = "cuda:0"
    ctx = chemk.Context(mech, device=0)
    # the DI reference and timing: the whole block, or a stratified sample
    if wl["di_cells"] and wl["di_cells"] < n:
        rng = np.random.default_rng(77)
        di_idx = np.sort(np.concatenate([rng.choice(np.nonzero(region == r)[0], wl["di_cells"] // 3,
                                                    replace=False) for r in range(3)]))
    else:
        di_idx = np.arange(n)
    nd = di_idx.size
    stock_counters = args.workload == "medium" and not args.weights   # the run the stored counters were taken on
    Tin = torch.from_numpy(T0).to(dev)
    Yin = torch.from_numpy(Y0).to(dev)
    P = torch.from_numpy(p0).to(dev)
    TinD = torch.from_numpy(T0[di_idx]).to(dev)
    YinD = torch.from_numpy(np.ascontiguousarray(Y0[di_idx])).to(dev)
    PD = torch.from_numpy(p0[di_idx]).to(dev)

    have_ann = False
    mode = args.mode
    if mode in ("auto", "ann"):
        try:
            from paper_2402_18858_amd import train
            if args.weights:
                train.load(ctx, args.weights)
                log(f"ann: loaded {args.weights}")
                have_ann = True
            else:
                have_ann = train.load_or_train(ctx, mech, dt, log=log, path=train.weights_path(mech))
        except Exception as e:  # noqa: BLE001 - reported, DI remains measurable
            log(f"ANN path unavailable ({e})")
            if mode == "ann":
                raise
        mode = "ann" if have_ann else "di"

    if args.species_only:
        if not have_ann or getattr(ctx, "species_nets", False):
            raise SystemExit("bench.py: --species-only takes its normalisation from a one-network weight file")
        sp = species_timing(ctx, mech, Tin, P, Yin, log)
        print(json.dumps({"metric": "per-species network forward", "value": sp["cells_per_s"],
                          "unit": "cell-forwards/s", "n_gpus": 1, "higher_is_better": True,
                          "dtype": "bf16", "data": "synthetic",
                          "config": {"workload": f"{n} cells ({wl['nx']}^3 flame block) x {K} species"},
                          "roofline": sp["roofline"],
                          "species_networks": sp}))
        return

    # DI tuning on the workload (untimed): bins x waves-per-CU grid on copies
    if args.bins > 0:
        best_bins, best_wpc, tune_ms = args.bins, args.wpc or 8, 0.0
    else:
        best_bins, best_wpc, tune_ms = ctx.autotune(TinD, PD, YinD, dt, chemk.default_opts(rtol=wl["rtol"], di_kernel=args.di_kernel))
    log(f"DI autotune -> bins={best_bins} waves/CU={best_wpc} ({tune_ms:.1f} ms)")

    def first_step(Ti, Pi, Yi, opts, k=1):
        """k eager steps, each from the initial state, with the phase timer on
        (HIP events around each phase's and each GEMM layer's launches on the
        step's stream): the accuracy reference and the phase split."""
        T, Y = Ti.clone(), Yi.clone()
        st = torch.zeros(Ti.numel(), dtype=torch.int32, device=dev)
        ns = torch.zeros(Ti.numel(), dtype=torch.int32, device=dev)
        ctx.timing(True)
        for _ in range(k):
            T.copy_(Ti)
            Y.copy_(Yi)
            ctx.advance(T, Pi, Y, dt, st, ns, opts=opts)
        ph = ctx.timing_read()
        ctx.timing(False)
        torch.cuda.synchronize()
        return T.cpu().numpy(), Y.cpu().numpy(), st.cpu().numpy(), ns.cpu().numpy(), ph

    def timed_graph(Ti, Pi, Yi, opts, k, w):
        """k steps, each on its own copy of the initial state made before the
        timed region, each replaying its captured graph (captured in the
        untimed warm-up, which also runs w extra steps)."""
        Ts = [Ti.clone() for _ in range(k)]
        Ys = [Yi.clone() for _ in range(k)]
        st = torch.zeros(Ti.numel(), dtype=torch.int32, device=dev)
        ns = torch.zeros(Ti.numel(), dtype=torch.int32, device=dev)
        for i in list(range(k)) + [j % k for j in range(w)]:
            ctx.advance(Ts[i], Pi, Ys[i], dt, st, ns, opts=opts)
        for i in range(k):
            Ts[i].copy_(Ti)
            Ys[i].copy_(Yi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(k):
            ctx.advance(Ts[i], Pi, Ys[i], dt, st, ns, opts=opts)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        del Ts, Ys
        return wall

    # ---- DI path -------------------------------------------------------------
    o_di = chemk.default_opts(bins=best_bins, waves_per_cu=best_wpc, rtol=wl["rtol"], di_kernel=args.di_kernel)
    o_di_g = chemk.default_opts(bins=best_bins, waves_per_cu=best_wpc, use_graph=1, rtol=wl["rtol"],
                                di_kernel=args.di_kernel)
    T_di, Y_di, st_di, ns_di, ph_di = first_step(TinD, PD, YinD, o_di)
    steps_total = float(ns_di.sum())
    di_kernel_ms = ph_di["di"][0] / max(ph_di["di"][1], 1)
    wall_di = timed_graph(TinD, PD, YinD, o_di_g, args.di_steps, 1)
    di_cups = nd * args.di_steps / wall_di
    fl_step = di_flops_per_step(K, mech.R)
    di_tflops = fl_step * steps_total / (di_kernel_ms * 1e-3) / 1e12
    di_info = {"cells": nd, "cell_updates_per_s": di_cups, "ms_per_step": 1e3 * wall_di / args.di_steps,
               "timed_steps": args.di_steps,
               "mean_rodas_steps_per_cell": steps_total / nd, "failed_cells": int((st_di != 0).sum()),
               "rodas_steps_per_cell_p50_p99_max": [float(np.percentile(ns_di, 50)),
                                                    float(np.percentile(ns_di, 99)), int(ns_di.max())],
               "kernel_ms": di_kernel_ms,
               "binning_ms": ph_di["binning"][0],
               "tuning": {"bins": best_bins, "waves_per_cu": best_wpc,
                          "di_kernel": ["auto", "lds_lu", "reg_lu"][args.di_kernel]},
               "rtol": o_di.rtol, "atol_Y": o_di.atol_Y}
    roof_di = {"bound": "alu", "achieved": di_tflops, "peak": PEAK_FP64_TFLOPS,
               "unit": "TFLOP/s", "frac": di_tflops / PEAK_FP64_TFLOPS,
               "traffic": measured_traffic("di_kernel") if stock_counters else None,
               "kernel": f"di_kernel (N = {K + 1})",
               "flops_per_rodas_step": fl_step, "rodas_steps": steps_total,
               "note": f"algorithmic FP64 count, exp/log = {EXP_FLOPS} operations"}
    log(f"DI ({nd} cells): {1e3 * wall_di / args.di_steps:.1f} ms per step, {di_cups:.4g} cell-updates/s")

    result = {"metric": "chem cell-updates/s (BF16 ANN vs FP64 DI), 262k cells x 32 sp; err vs oracle",
              "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "data": "synthetic",
              "unit": "cell-updates/s"}
    cfg = {"workload": f"{n} cells ({wl['nx']}^3 flame block) x {K} species / {mech.R} reactions, "
                       f"dt={dt:g} s", "cells": n, "species": K, "reactions": mech.R}
    if args.weights:
        cfg["weights"] = os.path.basename(args.weights)
    if mode == "di":
        result.update({"value": di_cups, "ms_per_step": 1e3 * wall_di / args.di_steps,
                       "steps": args.di_steps, "dtype": "f64",
                       "config": dict(cfg, path="DI (RODAS, FP64), hipGraph replays", di_cells=nd),
                       "roofline": roof_di, "di": di_info})
    else:
        o_ann = chemk.default_opts(mode=chemk.MODE_ANN, bins=best_bins, waves_per_cu=best_wpc,
                                   di_kernel=args.di_kernel,
                                   rtol=wl["rtol"])
        o_ann_g = chemk.default_opts(mode=chemk.MODE_ANN, bins=best_bins, waves_per_cu=best_wpc,
                                     di_kernel=args.di_kernel,
                                     use_graph=1, rtol=wl["rtol"])
        nsp = 5
        T_a, Y_a, st_a, ns_a, ph_a = first_step(Tin, P, Yin, o_ann, nsp)
        _, _, _, sd_y, _ = ctx.ann_get_norm()
        acc_ann = ann_vs_di(mech, sd_y, Y0[di_idx], T_a[di_idx], Y_a[di_idx], st_a[di_idx], T_di, Y_di,
                            chemk.CELL_ROUTED_DI)
        routed_all = (st_a & chemk.CELL_ROUTED_DI) != 0
        acc_ann.update({"cells_compared": nd, "routed_cells_block": int(routed_all.sum()),
                        "routed_fraction_block": float(routed_all.mean())})
        wall_a = timed_graph(Tin, P, Yin, o_ann_g, args.steps, args.warmup)
        cnt = ctx.last_counters()
        ann_cups = n * args.steps / wall_a
        dims = ctx.dims
        # per-species networks: K networks of these dims run together
        nets = K if getattr(ctx, "species_nets", False) else 1
        layer_fl = [2 * nets * dims[i] * dims[i + 1] for i in range(len(dims) - 1)]
        launches = {f"layer{i + 1}": ph_a[f"layer{i + 1}"] for i in range(min(4, len(dims) - 1))}
        per_layer = {}
        for i, (k_, (ms, nl)) in enumerate(launches.items()):
            rows = n * nsp / max(nl, 1)            # rows per launch (one MLP chunk)
            avg = ms / max(nl, 1)
            tf = layer_fl[i] * rows / (avg * 1e-3) / 1e12 if avg > 0 else 0.0
            per_layer[k_] = {"launches": nl, "avg_launch_us": 1e3 * avg, "rows_per_launch": rows,
                             "tflops": tf, "frac": tf / PEAK_BF16_TFLOPS}
        mlp_ms = ph_a["mlp"][0] / nsp
        mlp_tf = nets * train.mlp_flops_per_cell(dims) * n / (mlp_ms * 1e-3) / 1e12
        phases = {k_: {"ms_per_step": v[0] / nsp, "launches_per_step": v[1] / nsp}
                  for k_, v in ph_a.items() if v[1] > 0}
        # HBM streams of the ingest and post kernels, algorithmic bytes per cell
        ing_b = 8 * (K + 2) + 2 * 64 + 4 + 8          # T, p, Y in; X row, route, h0 out
        post_b = 8 * K + 4 * K + 4 + 8 + 8 + (8 * K + 8 + 4)   # Y, out, route, h0, T in; Y, T, status out
        hbm = {"ingest": {"bytes_per_cell": ing_b,
                          "GB_per_s": ing_b * n / (phases["ingest"]["ms_per_step"] * 1e-3) / 1e9},
               "post": {"bytes_per_cell": post_b,
                        "GB_per_s": post_b * n / (phases["post"]["ms_per_step"] * 1e-3) / 1e9},
               "peak_GB_per_s": PEAK_HBM_GBS}
        # the dominant kernel of the step: the DI fallback when it outweighs
        # the network's GEMMs, else the GEMM layer with the most work
        fb_ms = phases.get("fallback", {}).get("ms_per_step", 0.0)
        # (the layer with the most work: the phase timer's events inflate the
        # short layer-1 launches, so measured time would misname it)
        dom = max(per_layer, key=lambda k_: layer_fl[int(k_[-1]) - 1])
        roof_mlp = {"bound": "mfma", "achieved": per_layer[dom]["tflops"], "peak": PEAK_BF16_TFLOPS,
                    "unit": "TFLOP/s", "frac": per_layer[dom]["frac"],
                    "traffic": (measured_traffic("gemm_layer2") if (stock_counters and dom == "layer2")
                                else None),
                    "kernel": (f"gemm_dma_kernel, MLP {dom} ({dims[int(dom[-1]) - 1]} -> {dims[int(dom[-1])]}, "
                               f"{per_layer[dom]['rows_per_launch']:.0f} rows per launch)" if nets == 1 else
                               f"gemm_bf16_kernel grouped over {nets} per-species networks, {dom} "
                               f"({dims[int(dom[-1]) - 1]} -> {dims[int(dom[-1])]}, "
                               f"{per_layer[dom]['rows_per_launch']:.0f} rows per launch)"),
                    "flops_per_launch": layer_fl[int(dom[-1]) - 1] * per_layer[dom]["rows_per_launch"],
                    "mlp_phase": {"ms_per_step": mlp_ms, "tflops": mlp_tf,
                                  "frac": mlp_tf / PEAK_BF16_TFLOPS,
                                  "flops_per_cell": nets * train.mlp_flops_per_cell(dims)},
                    "per_layer": per_layer}
        routed_ns = ns_a[routed_all]
        fb_steps = float(routed_ns.sum()) * nsp
        if fb_ms > mlp_ms and fb_steps > 0:
            fb_tf = fl_step * routed_ns.sum() / (fb_ms * 1e-3) / 1e12
            roof = {"bound": "alu", "achieved": fb_tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                    "frac": fb_tf / PEAK_FP64_TFLOPS,
                    "traffic": (measured_traffic("di_kernel_routed", int(routed_all.sum()))
                                if stock_counters else None),
                    "kernel": f"di_kernel (N = {K + 1}) on the {int(routed_all.sum())} routed cells",
                    "flops_per_rodas_step": fl_step, "rodas_steps": float(routed_ns.sum()),
                    "mlp": roof_mlp}
        else:
            roof = roof_mlp
        result.update({"value": ann_cups, "ms_per_step": 1e3 * wall_a / args.steps,
                       "dtype": "bf16+f64",
                       "config": dict(cfg, path="ANN (BF16 MFMA) + DI fallback, hipGraph replays",
                                      di_cells=nd),
                       "roofline": roof, "di": di_info, "di_roofline": roof_di,
                       "ann": {"phases_eager": phases, "hbm_streams": hbm,
                               "routed_rodas_steps_p50_max": (
                                   [float(np.percentile(routed_ns, 50)), int(routed_ns.max())]
                                   if routed_ns.size else None),
                               "routed_cells_per_step": cnt["routed"],
                               "network_only_ms_per_step": sum(phases[k_]["ms_per_step"] for k_ in
                                                               ("ingest", "mlp", "post") if k_ in phases),
                               "speedup_over_di": ann_cups / di_cups, "error_vs_di": acc_ann}})
        log(f"ANN: {1e3 * wall_a / args.steps:.3f} ms per step, {ann_cups:.4g} cell-updates/s, "
            f"routed {int(routed_all.sum())}")
        result["closure"] = closure_timing(ctx, mech, Tin, P, Yin, T_a, Y_a, dt, log)
        if not args.no_species and nets == 1:
            try:   # a side measurement: it must not cost the headline line
                result["species_networks"] = species_timing(ctx, mech, Tin, P, Yin, log)
            except Exception as e:  # noqa: BLE001 - reported in the line
                log(f"per-species networks not timed ({e})")
                result["species_networks"] = {"error": str(e)}
        if args.envelope_sweep:
            result["ann"]["envelope_sweep"] = envelope_sweep(ctx, mech, dt, Tin, P, Yin, o_ann, region,
                                                             T_di, Y_di, sd_y, di_idx, log)

    # ---- CPU baseline: the oracle on bounded samples ----------------------------
    if not args.no_cpu_baseline and nd == n:
        import oracle
        rng = np.random.default_rng(99)
        om = oracle.OracleMech(mech)
        cores = oracle.default_threads()

        def sample(m):
            return np.sort(np.concatenate([rng.choice(np.nonzero(region == r)[0], m // 3,
                                                      replace=False) for r in range(3)]))

        idx = sample(args.cpu_sample)
        t0 = time.perf_counter()
        om.advance(T0[idx], p0[idx], Y0[idx], dt, rtol=o_di.rtol, atol_Y=o_di.atol_Y,
                   atol_T=o_di.atol_T, nthreads=cores)
        tc = time.perf_counter() - t0
        idr = sample(args.cpu_sample_ref)
        t0 = time.perf_counter()
        To, Yo = om.advance(T0[idr], p0[idr], Y0[idr], dt, nthreads=cores)[:2]
        tr = time.perf_counter() - t0
        big = Yo > 1e-8
        result["di_error_vs_oracle"] = {
            "cells": int(len(idr)), "oracle_rtol": 1e-10, "gpu_rtol": o_di.rtol,
            "max_rel_Y_above_1e-8": float((np.abs(Y_di[idr] - Yo)[big] / Yo[big]).max()),
            "max_abs_T_K": float(np.abs(T_di[idr] - To).max())}
        result["cpu_baseline"] = {
            "value": len(idx) / tc, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{len(idx)} cells stratified over the 3 regions of the same block, oracle "
                      f"DI at the GPU tolerance (rtol {o_di.rtol:g}), {tc:.1f} s",
            "value_reference_tolerance": len(idr) / tr,
            "sample_reference_tolerance": f"{len(idr)} cells, rtol 1e-10, {tr:.1f} s"}
    print(json.dumps(result))


if __name__ == "__main__":
    main()
