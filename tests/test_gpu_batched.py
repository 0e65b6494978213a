"""Batched dispatch on the GPU: every launch configuration (solver tile shape x launch mode,
solver form, staged predictor or fused predictor of each tile shape) gives the same bits,
the autotuner keeps a valid one, and a multi-step run captured in one HIP graph (per-patch
local dt, or guard exchange + global dt) reproduces the eager calls bitwise on every replay
and the oracle's run step for step."""
import numpy as np
import pytest

from gpu_util import dev, host, log, make_bunch, rel_err_fields
from paper_2508_09568_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ragged(seed_noise=0):
    w = W.uneven(mix=((9, 3), (13, 2), (20, 2)), nsteps=4)
    return w.layout, w.U.numpy().copy(), np.ascontiguousarray(w.dx), w.gamma


@pytest.mark.parametrize("case,precision", [("ragged3d", 8), ("ot64", 8), ("sod", 8),
                                            ("ragged3d", 4), ("ot64", 4), ("sod", 4)])
def test_every_launch_configuration_gives_identical_bits(case, precision):
    """In either precision every configuration gives the bits of every other; the common
    result is within the per-step bar of the oracle (FP64 1e-12; FP32 2e-5 against the
    oracle's update of the same FP32-rounded state)."""
    import oracle
    import torch
    log(f"[gpu] launch configurations case={case} precision={precision}")
    if case == "ragged3d":
        L, U, dx, gam = _ragged()
    elif case == "ot64":
        w = W.orszag_tang(64, 32)
        L, U, dx, gam = w.layout, w.U.copy(), w.dx, w.gamma
        oracle.fill_guards(U, L.dims, L.g, w.nbr)
    else:
        w = W.sod(128, patches=2)
        L, U, dx, gam = w.layout, w.U.copy(), w.dx, w.gamma
        oracle.fill_guards(U, L.dims, L.g, w.nbr)
    if precision == 4:
        U = U.astype(np.float32).astype(np.float64)
    prm = oracle.Params(gamma=gam)
    dt = oracle.cfl_many(U, L.dims, L.g, dx, prm)
    ref = oracle.step_many(U, L.dims, L.g, dt, dx, prm)
    B = make_bunch(L, gam, precision=precision)
    cfgs = B.tile_configs()
    assert len(cfgs) >= 2 and B.tile() == 0
    dty = torch.float64 if precision == 8 else torch.float32
    Ui, dtd, dxd = dev(U).to(dty), dev(dt), dev(dx)
    # every other patch at rest (dt = 0): copied, while the others match the full update
    dtm = dt.copy()
    dtm[::2] = 0.0
    dtmd = dev(dtm)
    expect = None
    outs = []
    modes = B.predictor_modes()
    assert len(modes) >= 2 and modes[0] == (0, 0, 0)
    for fused in range(len(modes)):
        B.set_predictor(fused)
        assert B.predictor() == fused
        for split in range(4):
            B.set_solver_split(split)
            assert B.solver_split() == split
            for i, cfg in enumerate(cfgs):
                B.set_tile(i)
                Uo = torch.zeros_like(Ui)
                B.update(Ui, Uo, dtd, dxd)
                assert B.check() == 0
                outs.append(host(Uo))
                log(f"    predictor {fused} split {split} config {i} {cfg}: max|diff| vs first = "
                    f"{np.abs(outs[-1] - outs[0]).max():.3e}")
                if expect is None:
                    expect = outs[0].copy()
                    for p in range(0, L.P, 2):
                        L.interior(expect, p)[...] = L.interior(U, p)
                Um = torch.zeros_like(Ui)
                B.update(Ui, Um, dtmd, dxd)
                assert B.check() == 0
                got = host(Um)
                for p in range(L.P):
                    assert np.array_equal(L.interior(got, p), L.interior(expect, p)), \
                        (fused, split, i, p)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    err = rel_err_fields(L, outs[0], ref)
    log(f"    {len(outs)} configurations; per-field rel err vs oracle {err}")
    assert err.max() <= (1e-12 if precision == 8 else 2e-5), err


def test_autotune_picks_a_configuration_and_keeps_results():
    log("[gpu] autotune on a ragged bunch")
    L, U, dx, gam = _ragged()
    import oracle
    dt = oracle.cfl_many(U, L.dims, L.g, dx, oracle.Params(gamma=gam))
    B = make_bunch(L, gam, precision=4)
    Ui, dtd, dxd = dev(U).float(), dev(dt), dev(dx)
    Uo = B.new_state()
    B.update(Ui, Uo, dtd, dxd)
    ref = host(Uo)
    best, ms = B.autotune(Ui, Uo, dtd, dxd, reps=2)
    log(f"    best {best} {B.tile_configs()[best]} ms {['%.3f' % m for m in ms]}")
    assert 0 <= best < len(ms) and B.tile() == best
    assert all(m > 0 for m in ms) and ms[best] == min(ms)
    assert 0 <= B.predictor() < len(B.predictor_modes())
    Uo.zero_()
    B.update(Ui, Uo, dtd, dxd)
    assert np.array_equal(host(Uo), ref)


@pytest.mark.parametrize("precision", [8, 4])
def test_graph_local_dt_run_matches_eager_calls_on_every_replay(precision):
    """4 steps, each patch at its own CFL step, frozen guards, ping-pong buffers."""
    import torch
    log(f"[gpu] graph-captured local-dt run, precision {precision}")
    L, U, dx, gam = _ragged()
    B = make_bunch(L, gam, precision=precision)
    dt_ = torch.float64 if precision == 8 else torch.float32
    U0 = dev(U).to(dt_)
    dxd = dev(dx)
    # eager reference
    a, b = U0.clone(), U0.clone()
    dte = torch.zeros(L.P, dtype=torch.float64, device="cuda")
    dts = []
    for k in range(4):
        B.cfl(a, dxd, dte, global_min=False)
        dts.append(host(dte).copy())
        B.update(a, b, dte, dxd)
        a, b = b, a
    eager = host(a)
    # graph: U_a holds the input, result of an even step count lands in U_a
    Ua, Ub = U0.clone(), U0.clone()
    dtg = torch.zeros(L.P, dtype=torch.float64, device="cuda")
    B.graph_capture(4, Ua, Ub, dtg, dxd, nbr=None, dt_mode=1)
    for rep in range(3):
        Ua.copy_(U0)
        Ub.copy_(U0)
        torch.cuda.synchronize()
        B.graph_launch()
        torch.cuda.synchronize()
        got = host(Ua)
        log(f"    replay {rep}: max|graph - eager| = {np.abs(got - eager).max():.3e}")
        assert np.array_equal(got, eager)
        assert np.array_equal(host(dtg), dts[-1])
        assert B.check() == 0
        # unrelated eager work between replays
        (U0 * 2).sum().item()
    if precision == 8:
        import oracle
        prm = oracle.Params(gamma=gam)
        Uo = U.copy()
        for k in range(4):
            d = oracle.cfl_many(Uo, L.dims, L.g, dx, prm)
            assert np.allclose(d, dts[k], rtol=1e-13, atol=0)
            Uo = oracle.step_many(Uo, L.dims, L.g, dts[k], dx, prm)
        err = rel_err_fields(L, eager, Uo)
        log(f"    4 local-dt steps vs oracle: {err.max():.2e}")
        assert err.max() <= 1e-11


def test_graph_with_guard_exchange_and_global_dt_matches_eager_calls():
    import torch
    log("[gpu] graph-captured run with guard fill and global dt (OT 64^2)")
    w = W.orszag_tang(64, 32)
    L = w.layout
    B = make_bunch(L, w.gamma)
    U0 = dev(w.U)
    dxd = dev(w.dx)
    nb = dev(w.nbr.astype(np.int32))
    a, b = U0.clone(), U0.clone()
    dte = torch.zeros(L.P, dtype=torch.float64, device="cuda")
    for k in range(5):
        B.fill_guards(a, nb)
        B.cfl(a, dxd, dte, global_min=True)
        B.update(a, b, dte, dxd)
        a, b = b, a
    eager = host(a)     # odd step count: result in the second buffer of the pair
    Ua, Ub = U0.clone(), U0.clone()
    dtg = torch.zeros(L.P, dtype=torch.float64, device="cuda")
    B.graph_capture(5, Ua, Ub, dtg, dxd, nbr=nb, dt_mode=2)
    for rep in range(2):
        Ua.copy_(U0)
        Ub.copy_(U0)
        B.graph_launch()
        got = host(Ub)
        assert np.array_equal(got, eager), rep
    assert B.check() == 0


def test_binding_rejects_mismatched_tensors():
    """The library sees plain pointers, so the binding checks every buffer: a wrong element
    type, count, layout or device raises before anything is launched."""
    import torch
    L, U, dx, gam = _ragged()
    B = make_bunch(L, gam)
    Ua, Ub = dev(U), dev(np.zeros_like(U))
    dt = torch.full((L.P,), 1e-4, dtype=torch.float64, device="cuda")
    dxd = dev(dx)
    nb = torch.zeros((L.P, 27), dtype=torch.int32, device="cuda")
    bad = [
        lambda: B.update(Ua, Ub, dt.float(), dxd),                     # dt in float32
        lambda: B.update(Ua, Ub, dt[:-1], dxd),                        # dt too short
        lambda: B.update(Ua, Ub, dt, dxd.t()),                         # dx not contiguous
        lambda: B.update(Ua.float(), Ub, dt, dxd),                     # state of the wrong type
        lambda: B.update(Ua[:-1], Ub[:-1], dt, dxd),                   # state too short
        lambda: B.update(Ua.cpu(), Ub, dt, dxd),                       # host tensor
        lambda: B.cfl(Ua, dxd[:-1], dt),
        lambda: B.fill_guards(Ua, nb.long()),                          # int64 neighbour table
        lambda: B.graph_capture(2, Ua, Ub, dt, dxd, nbr=nb[:-1]),
    ]
    for k, call in enumerate(bad):
        with pytest.raises(ValueError):
            call()
    torch.cuda.synchronize()
    B.update(Ua, Ub, dt, dxd)                                          # the handle still works
    assert B.check() == 0


def test_graph_capture_rejects_bad_arguments():
    import torch

    from paper_2508_09568_amd.binding import MhdError
    L, U, dx, gam = _ragged()
    B = make_bunch(L, gam)
    Ua = dev(U)
    dtg = torch.zeros(L.P, dtype=torch.float64, device="cuda")
    with pytest.raises(MhdError):
        B.graph_capture(2, Ua, Ua, dtg, dev(dx), dt_mode=1)
    with pytest.raises(MhdError):
        B.graph_launch()
