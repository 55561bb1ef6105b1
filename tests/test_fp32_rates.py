"""Measurement behind keeping the DI right-hand side in FP64: the oracle built
with FP32 rate products and production rates (rate constants from FP64
exp/log; Jacobian, LU, error control and the final enthalpy inversion in
FP64) against the FP64 oracle, both at the GPU's production tolerance, on
cells with a stored rtol-1e-10 reference.  FP32 rates miss the 1e-6 parity
bar on the 32-species flame block and cost extra steps on the 9-species
mechanism.  Oracle only (CPU); the variant is compiled here from
oracle/chem_oracle.c with -DOR_RATE_T=float."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from synth import mechanism as sm, workload as sw
from tests.gpu_util import announce

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")
PROD = dict(rtol=1e-7, atol_Y=1e-14, atol_T=1e-6)


@pytest.fixture(scope="module")
def fp32_lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("fp32r") / "liboracle_fp32r.so")
    src = os.path.join(os.path.dirname(HERE), "oracle", "chem_oracle.c")
    subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-fopenmp",
                           "-DOR_RATE_T=float", "-o", out, src, "-lm"])
    return oracle.load(out)


def _max_rel(Y, Yr):
    big = Yr > 1e-8
    return float((np.abs(Y - Yr)[big] / Yr[big]).max())


def test_fp32_rates_miss_the_parity_bar_on_the_flame_block(fp32_lib):
    mech = sm.mech_medium()
    g = np.load(os.path.join(GOLD, "di_medium_sample.npz"))
    T, p, Y, region = sw.flame_block(mech, 64, 2002)
    gi = np.nonzero(region[g["idx"]] == 2)[0][:48]       # product cells with a radical pool
    idx = g["idx"][gi]
    om64, om32 = oracle.OracleMech(mech), oracle.OracleMech(mech, library=fp32_lib)
    _, Y64, s64, n64 = om64.advance(T[idx], p[idx], Y[idx], 5e-7, **PROD)
    _, Y32, s32, n32 = om32.advance(T[idx], p[idx], Y[idx], 5e-7, **PROD)
    e64, e32 = _max_rel(Y64, g["Y"][gi]), _max_rel(Y32, g["Y"][gi])
    announce(f"FP32 rates, 32 species: max rel Y {e32:.2e} ({n32.mean():.0f} steps) vs FP64 "
             f"{e64:.2e} ({n64.mean():.0f} steps)")
    assert (s64 == 0).all() and e64 < 1e-6
    assert e32 > 1e-6


def test_fp32_rates_cost_steps_on_the_small_mechanism(fp32_lib):
    mech = sm.mech_small()
    g = np.load(os.path.join(GOLD, "di_small_4096.npz"))
    T, p, Y = sw.uniform_cells(mech, 4096, 2001)
    idx = np.arange(0, 4096, 16)
    om64, om32 = oracle.OracleMech(mech), oracle.OracleMech(mech, library=fp32_lib)
    _, Y64, _, n64 = om64.advance(T[idx], p[idx], Y[idx], 1e-6, **PROD)
    _, Y32, _, n32 = om32.advance(T[idx], p[idx], Y[idx], 1e-6, **PROD)
    e64, e32 = _max_rel(Y64, g["Y"][idx]), _max_rel(Y32, g["Y"][idx])
    announce(f"FP32 rates, 9 species: max rel Y {e32:.2e} ({n32.mean():.0f} steps) vs FP64 "
             f"{e64:.2e} ({n64.mean():.0f} steps)")
    assert e64 < 1e-6
    assert n32.mean() > 1.3 * n64.mean()
