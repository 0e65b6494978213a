"""The comparisons whose bars lie below what multiply-add contraction changes, run through the
parity build of the library (same sources; no contraction, correctly rounded division and
square root).  Started by test_gpu_parity_build.py in a process of its own with
MHD_PARITY_BUILD=1 (the binding then loads libmhdbunch_strict.so); prints the measured errors
as its last line (JSON)."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
sys.path.insert(0, os.path.dirname(HERE))


def main():
    if os.environ.get("MHD_PARITY_BUILD") != "1":
        raise SystemExit("run with MHD_PARITY_BUILD=1")
    from paper_2508_09568_amd import binding
    if not (binding.PARITY_BUILD and binding.LIB_PATH.endswith("libmhdbunch_strict.so")):
        raise SystemExit(f"the parity build is not loaded: {binding.LIB_PATH}")
    import test_gpu_adjoint as A
    import test_gpu_parity as P
    from gpu_util import log
    out = {"library": os.path.basename(binding.LIB_PATH)}
    for name in ("adjoint32", "turb3d", "ot64"):
        log(f"[parity build] step parity fp64 case={name}")
        err, plain = P.step_errors(name)
        out[f"step_{name}"] = {"r12": float(err.max()), "plain": float(plain.max())}
    for name in ("adjoint16", "ot32"):
        log(f"[parity build] adjoint dot-product case={name}")
        rel, guards_zero = A.dot_product_error(name)
        out[f"dot_{name}"] = {"rel": rel, "guards_zero": guards_zero}
    log("[parity build] adjoint configuration: 20 steps, checkpoint 5, 64^3")
    out["adjoint_case"] = A.adjoint_case_errors()
    print(json.dumps({"parity_build": out}), flush=True)


if __name__ == "__main__":
    main()
