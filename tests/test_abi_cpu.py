"""The C-ABI library loads, exports every declared symbol and validates
mechanisms and arguments on the host (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from synth import mechanism as sm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    txt = open(os.path.join(ROOT, "include", "chemk.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(chemk_[A-Za-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2402_18858_amd import chemk
    lib = C.CDLL(chemk.LIB_PATH)
    syms = _header_symbols()
    assert len(syms) >= 20
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing
    # the binding declares exactly the header's entry points
    assert sorted(chemk.exported_symbols()) == syms


def test_mechanism_accepts_generated_mechanisms():
    from paper_2402_18858_amd import chemk
    for f in (sm.mech_small, sm.mech_medium, sm.mech_large):
        mm = f()
        m = chemk.Mechanism(mm)
        assert (m.K, m.R, m.E) == (mm.K, mm.R, mm.E)


def _broken(kind):
    m = sm.mech_small()
    if kind == "balance":
        m.products = m.products.copy()
        j = 0
        # replace a product by a species with another element vector
        other = [k for k in range(m.K)
                 if not np.array_equal(m.composition[k], m.composition[m.products[j, 0]])][0]
        m.products[j, 0] = other
    elif kind == "index":
        m.reactants = m.reactants.copy()
        m.reactants[3, 0] = m.K
    elif kind == "nan":
        m.log_A = m.log_A.copy()
        m.log_A[5] = np.nan
    elif kind == "empty":
        m.reactants = m.reactants.copy()
        m.reactants[2, :] = -1
    elif kind == "atoms":
        m.composition = m.composition.copy()
        m.composition[0, :] = 0
    elif kind == "flag":
        m.third_body = m.third_body.copy()
        m.third_body[0] = 2
    return m


@pytest.mark.parametrize("kind", ["balance", "index", "nan", "empty", "atoms", "flag"])
def test_mechanism_rejects_bad_input(kind):
    from paper_2402_18858_amd import chemk
    with pytest.raises(chemk.ChemkError) as ei:
        chemk.Mechanism(_broken(kind))
    assert ei.value.code == chemk.E_MECH


def test_too_many_species_rejected():
    from paper_2402_18858_amd import chemk
    els = ["H"]
    K = 64
    m = sm.custom(els, [[1]] * K, [[3.5, 0, 0, 0, 0, 0, 0]] * K, [])
    with pytest.raises(chemk.ChemkError) as ei:
        chemk.Mechanism(m)
    assert ei.value.code == chemk.E_MECH


def test_default_options():
    from paper_2402_18858_amd import chemk
    o = chemk.default_opts()
    assert o.mode == chemk.MODE_DI and o.rtol == 1e-7 and o.atol_Y == 1e-14
    assert o.max_steps == 100000 and o.project == 1 and o.use_graph == 0
    with pytest.raises(AttributeError):
        chemk.default_opts(no_such_field=1)


def test_context_without_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2402_18858_amd import chemk
    with pytest.raises(chemk.ChemkError) as ei:
        chemk.Context(sm.mech_small())
    assert ei.value.code in (chemk.E_HIP, chemk.E_ARG)
