"""GPU parity at the sizes and precisions of the named workloads, through the C ABI:

* uneven batch (2000 x 16^3 + 1000 x 24^3 + 500 x 32^3 + 100 x 48^3, FP32, frozen guards):
  10 steps captured in one HIP graph, each patch at its own CFL step, in the autotuned launch
  configuration, against the FP64 oracle's 10 steps on sampled patches of every size;
* Orszag-Tang 256^2 as 8 x 8 patches of 32^2 to t = 0.5: FP64 per step (every step from the
  oracle's state and time step) and the end state of a free GPU run; FP32 over the whole run
  with the oracle's time steps fed in;
* turbulence 512^3 (4096 x 32^3, FP64): one update of every patch against the oracle;
* turbulence 128^3 (64 x 32^3, FP64): ten full steps (guard exchange, global time step,
  update), each from the oracle's state, and the end state of a free GPU run.

Bars: FP64 <= 1e-12 per step (per-field metric of gpu_util.rel_err_fields); FP32 L1 <= 1e-5
per field after the run (time steps of the FP32 run are its own, within ~1e-7 of the
oracle's, where a test says so)."""
import numpy as np
import pytest

from gpu_util import (dev, host, l1_rel_face_field, l1_rel_fields, log, make_bunch,
                      rel_err_fields)
from paper_2508_09568_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64_STEP_TOL = 1e-12
FP32_RUN_TOL = 1e-5


def _l1_patches(layout, A, B, patches):
    num = np.zeros(8)
    den = np.zeros(8)
    for p in patches:
        a = layout.interior(A, p).reshape(8, -1)
        b = layout.interior(B, p).reshape(8, -1)
        num += np.abs(a - b).sum(axis=1)
        den += np.abs(b).sum(axis=1)
    return num / np.where(den > 0, den, den[4])


def test_uneven_batch_fp32_graph_ten_local_steps_vs_oracle():
    import oracle
    import torch
    log("[gpu] uneven 3600 patches fp32: 10 graph-captured own-CFL steps vs fp64 oracle")
    w = W.uneven(device="cuda", dtype=torch.float32)
    L = w.layout
    B = make_bunch(L, w.gamma, precision=4, cfl=w.cfl)
    U0 = w.U
    dxd = dev(w.dx)
    Ua, Ub = U0.clone(), U0.clone()
    dt = torch.zeros(L.P, dtype=torch.float64, device="cuda")
    B.cfl(Ua, dxd, dt)
    best, _ = B.autotune(Ua, Ub, dt, dxd, reps=1)
    log(f"    tuned {B.tile_configs()[best]}, predictor {B.predictor()}, form {B.solver_split()}")
    B.graph_capture(10, Ua, Ub, dt, dxd, nbr=None, dt_mode=1)
    Ua.copy_(U0)
    Ub.copy_(U0)
    B.graph_launch()
    assert B.check() == 0
    got = host(Ua)                                   # even step count: result in U_a
    # oracle: the same initial state (rounded to FP32), sampled patches, own step each step
    U32 = U0.double().cpu().numpy()
    sizes = L.dims[:, 0]
    samples = []
    for n in (16, 24, 32, 48):
        idx = np.nonzero(sizes == n)[0]
        samples += [int(idx[0]), int(idx[len(idx) // 2]), int(idx[-1])]
    prm = oracle.Params(gamma=w.gamma, cfl=w.cfl)
    worst = np.zeros(8)
    worst_b = np.zeros(3)
    for p in samples:
        a, b = int(L.base[p]), int(L.base[p + 1])
        Lp = W.Layout(L.dims[p][None], L.g)
        Up = U32[a:b].copy()
        for _ in range(10):
            d = oracle.cfl_many(Up, Lp.dims, L.g, w.dx[p][None], prm)
            Up = oracle.step_many(Up, Lp.dims, L.g, d, w.dx[p][None], prm)
        worst = np.maximum(worst, l1_rel_fields(Lp, got[a:b], Up))
        worst_b = np.maximum(worst_b, l1_rel_face_field(Lp, got[a:b], Up))
    log(f"    sampled {len(samples)} patches, FP32 L1 rel err per field {worst}")
    log(f"    face field components relative to the field's L1 magnitude {worst_b}")
    # rho, momenta, E and B_x against their own L1 norms.  B_y and B_z are zero at t = 0
    # (uniform B along x) and after 10 steps only a small fraction of |B|; the rounding of the
    # EMF differences that create them is that of values of size |u||B|, so they are held to
    # the bar relative to the face field's magnitude, and their own-relative error to 3x it.
    assert np.all(worst[:6] <= FP32_RUN_TOL), worst
    assert np.all(worst_b <= FP32_RUN_TOL), worst_b
    assert np.all(worst[6:] <= 3 * FP32_RUN_TOL), worst


def _ot256():
    import oracle
    w = W.orszag_tang(256, 32)
    U = np.ascontiguousarray(w.U, dtype=np.float64).copy()
    oracle.fill_guards(U, w.layout.dims, w.layout.g, w.nbr)
    return w, U


def test_orszag_tang_256_fp64_every_step_and_end_state():
    import oracle
    import torch
    log("[gpu] Orszag-Tang 256^2 (8x8 x 32^2) fp64 to t=0.5: every step from the oracle's state")
    w, U = _ot256()
    L = w.layout
    prm = oracle.Params(gamma=w.gamma, cfl=w.cfl)
    B = make_bunch(L, w.gamma)
    dxd = dev(w.dx)
    nb = dev(w.nbr.astype(np.int32))
    dtd = torch.zeros(L.P, dtype=torch.float64, device="cuda")
    Ui = dev(U)
    Uo = torch.zeros_like(Ui)
    t, k, worst, dts = 0.0, 0, np.zeros(8), []
    Ur = U.copy()
    while t < 0.5 * (1 - 1e-14):
        oracle.fill_guards(Ur, L.dims, L.g, w.nbr)
        d = float(oracle.cfl_many(Ur, L.dims, L.g, w.dx, prm).min())
        d = min(d, 0.5 - t)
        nxt = oracle.step_many(Ur, L.dims, L.g, np.full(L.P, d), w.dx, prm)
        Ui.copy_(torch.as_tensor(Ur))
        B.fill_guards(Ui, nb)
        B.cfl(Ui, dxd, dtd, global_min=True)
        gd = float(host(dtd)[0])
        if d < 0.5 - t:
            assert abs(gd / d - 1.0) <= 1e-13, (k, gd, d)
        dtd.fill_(d)
        B.update(Ui, Uo, dtd, dxd)
        worst = np.maximum(worst, rel_err_fields(L, host(Uo), nxt))
        Ur = nxt
        t = 0.5 if d >= 0.5 - t else t + d
        k += 1
        dts.append(d)
    assert B.check() == 0
    oracle.fill_guards(Ur, L.dims, L.g, w.nbr)
    log(f"    {k} steps, worst per-step per-field rel err {worst}")
    assert np.all(worst <= FP64_STEP_TOL), worst
    # a free GPU run (its own guard exchange and global time step) to the same time
    Ua, Ub = dev(U), torch.zeros_like(Ui)
    t, kk = 0.0, 0
    while t < 0.5 * (1 - 1e-14):
        B.fill_guards(Ua, nb)
        B.cfl(Ua, dxd, dtd, global_min=True)
        d = min(float(host(dtd)[0]), 0.5 - t)
        dtd.fill_(d)
        B.update(Ua, Ub, dtd, dxd)
        Ua, Ub = Ub, Ua
        t = 0.5 if d >= 0.5 - t else t + d
        kk += 1
    B.fill_guards(Ua, nb)
    assert B.check() == 0 and kk == k
    end = rel_err_fields(L, host(Ua), Ur)
    log(f"    free GPU run end state vs oracle: per-field rel err {end}")
    assert np.all(end <= 1e-10), end


def test_orszag_tang_256_fp32_run_against_fp64_oracle():
    import oracle
    import torch
    log("[gpu] Orszag-Tang 256^2 fp32 to t=0.5 with the oracle's time steps")
    w, U = _ot256()
    L = w.layout
    prm = oracle.Params(gamma=w.gamma, cfl=w.cfl)
    U32 = U.astype(np.float32).astype(np.float64)
    ref, dref = oracle.run(U32, L.dims, L.g, w.dx, w.nbr, prm, t_end=0.5, record_dt=True)
    B = make_bunch(L, w.gamma, precision=4)
    dxd = dev(w.dx)
    nb = dev(w.nbr.astype(np.int32))
    dtd = torch.zeros(L.P, dtype=torch.float64, device="cuda")
    Ua = dev(U32).float()
    Ub = torch.zeros_like(Ua)
    for d in dref:
        B.fill_guards(Ua, nb)
        dtd.fill_(float(d))
        B.update(Ua, Ub, dtd, dxd)
        Ua, Ub = Ub, Ua
    B.fill_guards(Ua, nb)
    assert B.check() == 0
    l1 = l1_rel_fields(L, host(Ua), ref)
    log(f"    {len(dref)} steps, FP32 L1 rel err per field {l1}")
    assert np.all(l1 <= FP32_RUN_TOL), l1


@pytest.mark.timeout(900)
def test_turbulence_512_one_update_of_every_patch_fp64():
    """The whole 512^3 workload (4096 x 32^3): guard exchange, global time step and one
    update on the GPU against the oracle's on every patch (OpenMP over patches on the host)."""
    import time

    import oracle
    import torch
    log("[gpu] turbulence 512^3 fp64: one update of all 4096 patches vs oracle")
    t0 = time.perf_counter()
    w = W.turbulence(device="cuda")
    L = w.layout
    Ur = w.U.cpu().numpy()          # the generator's state for the oracle, before any launch
    prm = oracle.Params(gamma=w.gamma, cfl=w.cfl)
    B = make_bunch(L, w.gamma, cfl=w.cfl)
    Ui = w.U
    dxd = dev(w.dx)
    B.fill_guards(Ui, dev(w.nbr.astype(np.int32)))
    dtd = torch.zeros(L.P, dtype=torch.float64, device="cuda")
    B.cfl(Ui, dxd, dtd, global_min=True)
    Uo = torch.empty_like(Ui)
    best, _ = B.autotune(Ui, Uo, dtd, dxd, reps=1)
    log(f"    tuned {B.tile_configs()[best]}, predictor {B.predictor()}, form {B.solver_split()}")
    B.update(Ui, Uo, dtd, dxd)
    assert B.check() == 0
    gdt = float(host(dtd)[0])
    got = Uo.cpu().numpy()
    del Uo
    log(f"    GPU done ({time.perf_counter() - t0:.1f} s); oracle guard fill, time step, update")
    del Ui, w.U
    torch.cuda.empty_cache()
    oracle.fill_guards(Ur, L.dims, L.g, w.nbr)
    d = float(oracle.cfl_many(Ur, L.dims, L.g, w.dx, prm).min())
    assert abs(gdt / d - 1.0) <= 1e-13, (gdt, d)
    ref = oracle.step_many(Ur, L.dims, L.g, np.full(L.P, gdt), w.dx, prm)
    log(f"    oracle done ({time.perf_counter() - t0:.1f} s); comparing")
    err = rel_err_fields(L, got, ref)
    log(f"    all 4096 patches: per-field rel err {err} ({time.perf_counter() - t0:.1f} s)")
    assert np.all(err <= FP64_STEP_TOL), err


def test_turbulence_128_ten_full_steps_fp64():
    import oracle
    import torch
    log("[gpu] turbulence 128^3 (64 x 32^3) fp64: 10 full steps, each from the oracle's state")
    w = W.turbulence(N=128, patch=32)
    L = w.layout
    prm = oracle.Params(gamma=w.gamma, cfl=w.cfl)
    U0 = w.U.numpy().copy()
    B = make_bunch(L, w.gamma, cfl=w.cfl)
    dxd = dev(w.dx)
    nb = dev(w.nbr.astype(np.int32))
    dtd = torch.zeros(L.P, dtype=torch.float64, device="cuda")
    Ui = dev(U0)
    Uo = torch.zeros_like(Ui)
    Ur = U0.copy()
    worst = np.zeros(8)
    for k in range(10):
        Ui.copy_(torch.as_tensor(Ur))           # the oracle's state, its guards not yet filled
        oracle.fill_guards(Ur, L.dims, L.g, w.nbr)
        d = float(oracle.cfl_many(Ur, L.dims, L.g, w.dx, prm).min())
        nxt = oracle.step_many(Ur, L.dims, L.g, np.full(L.P, d), w.dx, prm)
        B.fill_guards(Ui, nb)
        B.cfl(Ui, dxd, dtd, global_min=True)
        assert abs(float(host(dtd)[0]) / d - 1.0) <= 1e-13, k
        assert np.array_equal(host(Ui), Ur), k            # guard exchange bitwise
        dtd.fill_(d)
        B.update(Ui, Uo, dtd, dxd)
        worst = np.maximum(worst, rel_err_fields(L, host(Uo), nxt))
        Ur = nxt
    assert B.check() == 0
    log(f"    worst per-step per-field rel err {worst}")
    assert np.all(worst <= FP64_STEP_TOL), worst
    # free GPU run of the same 10 steps
    Ua, Ub = dev(U0), torch.zeros_like(Ui)
    for k in range(10):
        B.fill_guards(Ua, nb)
        B.cfl(Ua, dxd, dtd, global_min=True)
        B.update(Ua, Ub, dtd, dxd)
        Ua, Ub = Ub, Ua
    assert B.check() == 0
    end = rel_err_fields(L, host(Ua), Ur)
    log(f"    free GPU run after 10 steps vs oracle: per-field rel err {end}")
    assert np.all(end <= 1e-11), end
