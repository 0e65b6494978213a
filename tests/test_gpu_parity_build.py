"""The parity build of the library (libmhdbunch_strict.so: the same sources without
multiply-add contraction and with correctly rounded division and square root, so every
operation rounds as the oracle's plain evaluation does) against the oracle at the bars that
contraction alone would break.  The comparisons run in a process of their own
(parity_build_child.py, MHD_PARITY_BUILD=1), since the binding loads one library per process.

Bars: one FP64 update within 1e-12 of the oracle in the plain per-field relative max-norm,
also on the adjoint configuration's degenerate background (the product library needs the
natural-scale floor of reading R12 there); the adjoint's dot-product identity within 1e-11 on
that background, whose HLLD star-state denominator amplifies rounding ~1e4 (measured 1.4e-12,
as a CPU build of the same code without contraction gives), 1e-12 elsewhere.  The 20-step
gradient of the adjoint configuration keeps the product library's 1e-6 bars: it differs from
the oracle's by ~3e-8 in both builds, the rollout's conditioning at the degenerate point, not
contraction."""
import json
import os
import subprocess
import sys

import pytest

from gpu_util import log

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_parity_build_against_oracle():
    env = dict(os.environ, MHD_PARITY_BUILD="1")
    log("[gpu] parity build: step parity, adjoint dot products, adjoint configuration")
    r = subprocess.run([sys.executable, "-u", os.path.join(HERE, "parity_build_child.py")],
                       env=env, capture_output=True, text=True, timeout=900)
    log(r.stdout[-6000:])
    assert r.returncode == 0, r.stderr[-6000:]
    line = [ln for ln in r.stdout.splitlines() if ln.startswith('{"parity_build"')][-1]
    res = json.loads(line)["parity_build"]
    assert res["library"] == "libmhdbunch_strict.so"
    for name in ("adjoint32", "turb3d", "ot64"):
        e = res[f"step_{name}"]
        assert e["plain"] <= 1e-12 and e["r12"] <= 1e-12, (name, e)
    assert res["dot_adjoint16"]["rel"] <= 1e-11 and res["dot_adjoint16"]["guards_zero"]
    assert res["dot_ot32"]["rel"] <= 1e-12 and res["dot_ot32"]["guards_zero"]
    a = res["adjoint_case"]
    assert a["guards_zero"] and a["clean"]
    assert a["directional"] <= 1e-6 and a["fd"] <= 1e-6 and a["duals"] <= 1e-6, a
