"""Wave-convergence check of the device code (CPU only: compiles to IR).

Every kernel of the library must keep cross-lane operations out of loops and
branches whose control depends on the lane; the checker itself is pinned on
small kernels with a known answer (tests/fixtures/convergence_cases.hip)."""
import os
import shutil
from concurrent.futures import ThreadPoolExecutor

import pytest

from tests import convergence_check as cc

pytestmark = pytest.mark.skipif(not os.path.exists(cc.HIPCC) and not shutil.which("hipcc"),
                                reason="hipcc not available")
HERE = os.path.dirname(os.path.abspath(__file__))


def _ir(src, tmp_path):
    out = str(tmp_path / (os.path.basename(src) + ".ll"))
    return open(cc.emit_ir(src, out)).read()


def test_checker_flags_known_bad_shapes(tmp_path):
    text = _ir(os.path.join(HERE, "fixtures", "convergence_cases.hip"), tmp_path)
    names = {f: cc.check_function(text, f) for f in cc.functions(text)}

    def found(key):
        return [x for f, v in names.items() if key in f for x in v]

    assert found("claim_lane0_branch"), "lane-0 claim loop not flagged"
    assert not found("claim_all_lanes"), found("claim_all_lanes")
    assert found("exit_on_butterfly"), "loop exiting on a butterfly sum not flagged"
    assert not found("exit_on_broadcast"), found("exit_on_broadcast")
    assert not found("exit_on_ballot"), found("exit_on_ballot")


def test_library_kernels_keep_waves_converged(tmp_path):
    srcs = [os.path.join(cc.CSRC, f) for f in sorted(os.listdir(cc.CSRC)) if f.endswith(".hip")]
    assert srcs
    with ThreadPoolExecutor(max_workers=4) as ex:
        texts = list(ex.map(lambda s: _ir(s, tmp_path), srcs))
    findings = [x for t in texts for x in cc.check_ir(t)]
    assert not findings, "\n".join(findings)
