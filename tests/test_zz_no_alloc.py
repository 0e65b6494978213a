"""The allocation-free update (mhd_bunch_update_static, through the C ABI) against the
update with the bound workspace's scratch: identical bits on two calls in a row (the second
with a smaller bunch sharing the same static array), in several launch configurations, and a
clear error when one chunk of patches does not fit the static scratch."""
import numpy as np
import pytest

from gpu_util import dev, host, log, make_bunch, rel_err_fields
from paper_2508_09568_amd import workloads as W

pytestmark = pytest.mark.gpu


def _turbulence_case(N, patch, precision):
    import torch

    import oracle
    w = W.turbulence(N=N, patch=patch)
    L = w.layout
    U = w.U.numpy().copy()
    if precision == 4:
        U = U.astype(np.float32).astype(np.float64)
    oracle.fill_guards(U, L.dims, L.g, w.nbr)
    prm = oracle.Params(gamma=w.gamma, cfl=w.cfl)
    dt = np.full(L.P, oracle.cfl_many(U, L.dims, L.g, w.dx, prm).min())
    dty = torch.float64 if precision == 8 else torch.float32
    return w, L, U, dt, dev(U).to(dty), dev(dt), dev(w.dx)


def _compare(w, L, Ui, dtd, dxd, precision, cap, configs):
    """update_static of a bunch capped at `cap` scratch bytes vs the plain update of an
    uncapped bunch, in each (predictor, solver form) of `configs`; returns the static result."""
    import torch

    from paper_2508_09568_amd.binding import STATIC_SCRATCH_BYTES
    Bs = make_bunch(L, w.gamma, precision=precision, max_scratch_bytes=cap)
    Bw = make_bunch(L, w.gamma, precision=precision)
    assert Bs.workspace.numel() <= cap + (64 << 20) and cap <= STATIC_SCRATCH_BYTES
    got = None
    for pred, split in configs:
        for B in (Bs, Bw):
            B.set_predictor(pred)
            B.set_solver_split(split)
        Uw = torch.full_like(Ui, float("nan"))
        Us = torch.full_like(Ui, float("nan"))
        Bw.update(Ui, Uw, dtd, dxd)
        Bs.update_static(Ui, Us, dtd, dxd)
        assert Bw.check() == 0 and Bs.check() == 0
        a, b = host(Uw), host(Us)
        for p in range(L.P):
            assert np.array_equal(L.interior(a, p), L.interior(b, p)), (pred, split, p)
        log(f"    predictor {pred} solver form {split}: identical bits on {L.P} patches")
        got = b
    return got


def test_static_update_matches_workspace_update_twice_second_smaller():
    import oracle
    log("[gpu] update_static: 128^3 FP64 (64 patches of 32^3), then 32^3 FP32 (8 of 16^3)")
    # first call: 64 patches of 32^3 in FP64 need ~1 GiB of scratch in all; capped at the
    # static size they run in chunks of 7 patches
    w, L, U, dt, Ui, dtd, dxd = _turbulence_case(128, 32, 8)
    got = _compare(w, L, Ui, dtd, dxd, 8, 128 << 20, [(0, 0), (1, 2), (1, 3), (2, 1)])
    prm = oracle.Params(gamma=w.gamma, cfl=w.cfl)
    some = [0, 21, 63]
    ref = oracle.step_many(U, L.dims, L.g, dt, w.dx, prm)
    err = rel_err_fields(L, got, ref, patches=some).max()
    log(f"    vs oracle on patches {some}: {err:.2e}")
    assert err <= 1e-12
    # second call, smaller bunch and other precision, on the same static array
    w, L, U, dt, Ui, dtd, dxd = _turbulence_case(32, 16, 4)
    _compare(w, L, Ui, dtd, dxd, 4, 8 << 20, [(0, 0), (1, 0)])


def test_static_update_rejects_a_chunk_beyond_the_static_scratch():
    """One 80^3 FP64 patch needs ~224 MiB of scratch, more than the static array holds:
    the call returns MHD_EINVAL before any launch and leaves the output untouched."""
    import torch

    from paper_2508_09568_amd.binding import MHD_EINVAL, MhdError
    dims = np.array([[80, 80, 80]], dtype=np.int32)
    from paper_2508_09568_amd.binding import Bunch
    B = Bunch(dims, g=3, precision=8)
    U = B.new_state()
    Uo = torch.full_like(U, 7.0)
    dt = dev(np.zeros(1))
    dx = dev(np.full((1, 3), 1.0 / 80))
    with pytest.raises(MhdError) as ei:
        B.update_static(U, Uo, dt, dx)
    assert ei.value.code == MHD_EINVAL and "static scratch" in str(ei.value)
    assert bool((Uo == 7.0).all())
