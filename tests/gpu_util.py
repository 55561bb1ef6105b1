"""Helpers shared by the GPU tests (device tensors, contexts)."""
import sys

import numpy as np


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def element_mass(mech, Y):
    """Element mass fractions (n, E) of mass fractions Y (n, K)."""
    comp = mech.composition.astype(np.float64)
    W = comp @ mech.element_mass
    Em = (comp * mech.element_mass[None, :]) / W[:, None]      # (K, E)
    return Y @ Em
