"""Write the oracle's expected DI results used by the GPU parity tests.

Calls only the oracle (and the seeded input generators); nothing here comes
from the GPU path.  Reference tolerance: rtol 1e-10, atol_Y 1e-18,
atol_T 1e-8 K (RODAS with step control, then element projection and T from
the conserved enthalpy).

    python tests/golden/make_golden.py [small|medium|large|all]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synth import mechanism as sm, workload as sw  # noqa: E402

REF = dict(rtol=1e-10, atol_Y=1e-18, atol_T=1e-8)


def medium_sample_index(om, T, p, Y, region, seed=4242, per_region=512, candidates=2048,
                        stiffest=1024):
    """Cells of the 64^3 block with an oracle reference: `per_region` drawn
    uniformly from each of the three regions, plus the `stiffest` cells (most
    oracle steps at rtol 1e-7) among `candidates` more drawn per region, so
    that the sample weights the stiffest cells, where the integrators' errors
    are largest."""
    rng = np.random.default_rng(seed)
    uni = np.concatenate([rng.choice(np.nonzero(region == r)[0], per_region, replace=False)
                          for r in range(3)])
    rest = np.setdiff1d(np.arange(T.size), uni)
    cand = np.concatenate([rng.choice(rest[region[rest] == r], candidates, replace=False)
                           for r in range(3)])
    ns = om.advance(T[cand], p[cand], Y[cand], 5e-7, rtol=1e-7, atol_Y=1e-14, atol_T=1e-6)[3]
    stiff = cand[np.argsort(-ns, kind="stable")[:stiffest]]
    return np.sort(np.concatenate([uni, stiff])), ns


def small():
    om = oracle.OracleMech(sm.mech_small())
    T, p, Y = sw.uniform_cells(om.src, 4096, 2001)
    t = time.time()
    T1, Y1, st, ns = om.advance(T, p, Y, 1e-6, **REF)
    print(f"small: {time.time() - t:.1f} s, steps mean {ns.mean():.0f}, status max {st.max()}")
    np.savez_compressed(os.path.join(HERE, "di_small_4096.npz"), T=T1, Y=Y1, status=st, nsteps=ns,
                        dt=1e-6, **{k: v for k, v in REF.items()})


def medium():
    om = oracle.OracleMech(sm.mech_medium())
    T, p, Y, region = sw.flame_block(om.src, 64, 2002)
    t = time.time()
    idx, ns_c = medium_sample_index(om, T, p, Y, region)
    print(f"medium: sample of {idx.size} cells chosen in {time.time() - t:.1f} s (candidate steps "
          f"median {np.median(ns_c):.0f}, max {ns_c.max()})")
    t = time.time()
    T1, Y1, st, ns = om.advance(T[idx], p[idx], Y[idx], 5e-7, **REF)
    print(f"medium: {time.time() - t:.1f} s, steps mean {ns.mean():.0f}, status max {st.max()}")
    np.savez_compressed(os.path.join(HERE, "di_medium_sample.npz"), idx=idx, T=T1, Y=Y1,
                        status=st, nsteps=ns, dt=5e-7, **{k: v for k, v in REF.items()})


def large(per_region=128):
    """The 53-species mechanism on its 128^3 block (2,097,152 cells): a
    stratified sample of the oracle's reference results."""
    om = oracle.OracleMech(sm.mech_large())
    T, p, Y, region = sw.flame_block(om.src, 128, 2005)
    rng = np.random.default_rng(4343)
    idx = np.sort(np.concatenate([rng.choice(np.nonzero(region == r)[0], per_region, replace=False)
                                  for r in range(3)]))
    t = time.time()
    T1, Y1, st, ns = om.advance(T[idx], p[idx], Y[idx], 5e-7, **REF)
    print(f"large: {idx.size} cells in {time.time() - t:.1f} s, steps mean {ns.mean():.0f}, "
          f"status max {st.max()}")
    np.savez_compressed(os.path.join(HERE, "di_large_sample.npz"), idx=idx, T=T1, Y=Y1,
                        status=st, nsteps=ns, dt=5e-7, **{k: v for k, v in REF.items()})


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("small", "all"):
        small()
    if which in ("medium", "all"):
        medium()
    if which in ("large", "all"):
        large()
