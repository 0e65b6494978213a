"""GPU local time stepping (mhd_bunch_lts_step) against the oracle: one step's guard fill
at each patch's own time, slice bookkeeping and time advance (bitwise, both precisions),
and whole runs with fixed per-patch steps, time levels and each patch's own CFL step (2D with
floating-point ties between symmetric patches, 3D without symmetry: the oracle's schedule)."""
import numpy as np
import pytest

from gpu_util import dev, host, log, make_bunch, rel_err_fields
from paper_2508_09568_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ot(patch=16):
    import oracle
    w = W.orszag_tang(64, patch)
    U = w.U.copy()
    oracle.fill_guards(U, w.layout.dims, w.layout.g, w.nbr)
    return w, U


@pytest.mark.parametrize("precision", [8, 4])
def test_one_step_fill_and_bookkeeping_match_oracle_bitwise(precision):
    import oracle
    import torch
    log(f"[gpu] lts one step, precision {precision}")
    w, U = _ot()
    L = w.layout
    rng = np.random.default_rng(7)
    t = rng.uniform(0.0, 1.0, L.P)
    tp = t - np.where(rng.uniform(size=L.P) < 0.8, rng.uniform(0.1, 0.5, L.P), 0.0)
    t[3] = t[3] + 5.0                                     # one patch past t_end
    # an earlier slice within 0.1 % (the weights reach |th| ~ 10 here: the update after the
    # fill must still see a physical state)
    Up = U * (1.0 + 1e-3 * rng.standard_normal(U.shape))
    if precision == 4:
        U = U.astype(np.float32).astype(np.float64)
        Up = Up.astype(np.float32).astype(np.float64)
    t_end = 2.0
    ready = oracle.lts_ready(t, t_end, w.nbr)
    assert 0 < ready.sum() < L.P
    ref = U.copy()
    oracle.fill_guards_at(ref, Up, t, tp, L.dims, L.g, w.nbr, mask=ready)
    B = make_bunch(L, w.gamma, precision=precision)
    dty = torch.float64 if precision == 8 else torch.float32
    Uc, Un, Upd = dev(U).to(dty), dev(np.zeros_like(U)).to(dty), dev(Up).to(dty)
    td, tpd, dtd = dev(t), dev(tp), dev(np.zeros(L.P))
    dtf = dev(np.full(L.P, 1e-5))
    B.lts_step(Uc, Un, Upd, td, tpd, dtd, dev(w.dx), dev(w.nbr.astype(np.int32)), t_end,
               dt_fixed=dtf)
    assert B.check() == 0
    want = ref.astype(np.float32) if precision == 4 else ref
    got = host(Uc)
    Uin = U.astype(want.dtype)
    for p in range(L.P):                                  # patches at rest untouched
        if not ready[p]:
            assert np.array_equal(L.view(got, p), L.view(Uin, p)), p
    guard = np.ones(L.total, dtype=bool)
    for p in range(L.P):
        L.interior(guard, p)[...] = False
    rmask = np.repeat(ready, np.diff(L.base))
    assert np.array_equal(got[guard & rmask], want[guard & rmask])   # interpolated guards
    assert not np.array_equal(got[~guard & rmask], Uin[~guard & rmask])  # interiors advanced
    dt_want = np.where(ready, np.minimum(1e-5, t_end - t), 0.0)
    if precision == 8:                                    # ... by the update of the filled state
        adv = oracle.step_many(ref, L.dims, L.g, dt_want, w.dx, oracle.Params(gamma=w.gamma))
        err = rel_err_fields(L, got, adv, patches=np.nonzero(ready)[0])
        assert err.max() <= 1e-12, err
    assert np.array_equal(host(dtd), dt_want)
    assert np.array_equal(host(tpd), np.where(ready, t, tp))
    assert np.array_equal(host(td), np.where(ready & (dt_want >= t_end - t), t_end, t + dt_want))
    # previous slice: a ready patch's owned values before the update (its guard cells are not
    # written: the guard fill reads owned values only); patches at rest untouched
    gp = host(Upd)
    Upw = Up.astype(want.dtype)
    for p in range(L.P):
        if ready[p]:
            assert np.array_equal(L.interior(gp, p), L.interior(want, p)), p
        else:
            assert np.array_equal(L.view(gp, p), L.view(Upw, p)), p
    assert np.array_equal(gp[guard], Upw[guard])


def test_run_with_fixed_steps_matches_oracle_driver():
    """Steps in powers of two by patch: exact time sums, so both sides take the same schedule
    (the same ready patches at every step) and the states agree to rounding."""
    import oracle
    from paper_2508_09568_amd import lts
    log("[gpu] lts run vs oracle, fixed per-patch steps")
    w, U = _ot()
    L = w.layout
    prm = oracle.Params(gamma=w.gamma)
    dtf = 1e-3 * 2.0 ** -(np.arange(L.P) % 3)
    t_end = 4e-3
    Uo, to, cnt, ns = oracle.lts_run(U, L.dims, L.g, w.dx, w.nbr, prm, t_end=t_end, dt_fixed=dtf)
    B = make_bunch(L, w.gamma)
    Ug, tg, n, cg = lts.run(B, dev(U), dev(w.dx), dev(w.nbr.astype(np.int32)), t_end,
                            dt_fixed=dev(dtf), check_every=1)
    assert B.check() == 0
    assert n == ns and np.array_equal(host(cg), cnt) and np.array_equal(host(tg), to)
    err = rel_err_fields(L, host(Ug), Uo)
    log(f"    {ns} steps, updates per patch {cnt.min()}..{cnt.max()}: rel err {err.max():.2e}")
    assert err.max() <= 1e-12 * cnt.max(), err


def test_run_with_own_cfl_steps_is_a_valid_schedule_close_to_the_oracle():
    """Each patch at its own CFL step.  Patches related by the Orszag-Tang symmetry have equal
    steps in exact arithmetic; whether they tie in floating point differs between the two
    implementations, and a tie decides whether two patches advance in one step or in two.
    So the step count is not unique: check what is (every patch ends at t_end, within one
    update of the oracle's count).  The states still agree to rounding: a patch advances only
    when no neighbour is behind it, so a neighbour at the same time that went first has that
    time as its previous slice and the guards interpolated from it are that slice exactly."""
    import oracle
    from paper_2508_09568_amd import lts
    log("[gpu] lts run vs oracle, own CFL steps")
    w, U = _ot()
    L = w.layout
    prm = oracle.Params(gamma=w.gamma)
    t_end = 0.02
    Uo, to, cnt, ns = oracle.lts_run(U, L.dims, L.g, w.dx, w.nbr, prm, t_end=t_end)
    B = make_bunch(L, w.gamma)
    Ug, tg, n, cg = lts.run(B, dev(U), dev(w.dx), dev(w.nbr.astype(np.int32)), t_end,
                            check_every=1)
    assert B.check() == 0
    assert np.all(host(tg) == t_end) and np.all(to == t_end)
    assert np.abs(host(cg) - cnt).max() <= 1
    G = host(Ug)
    num = sum(np.abs(L.interior(G, p) - L.interior(Uo, p)).sum() for p in range(L.P))
    den = sum(np.abs(L.interior(Uo, p)).sum() for p in range(L.P))
    log(f"    steps {n} vs {ns}; L1 rel difference {num / den:.2e}")
    assert num / den < 1e-12


def test_time_levels_match_oracle_driver():
    """Steps rounded down to a power-of-two quantum x 2^k: from the same (non-dyadic) per-patch
    steps both sides pick the same levels, so the schedule is identical and the states agree
    to rounding; the finest level sets the number of steps."""
    import oracle
    from paper_2508_09568_amd import lts
    log("[gpu] lts run vs oracle, time levels")
    w, U = _ot()
    L = w.layout
    prm = oracle.Params(gamma=w.gamma)
    own = oracle.cfl_many(U, L.dims, L.g, w.dx, prm)
    q = 2.0 ** np.floor(np.log2(0.7 * float(own.min())))
    dtf = own * np.linspace(1.0, 3.0, L.P)
    Uo, to, cnt, ns = oracle.lts_run(U, L.dims, L.g, w.dx, w.nbr, prm, t_end=8 * q,
                                     dt_fixed=dtf, dt_quantum=q)
    B = make_bunch(L, w.gamma)
    Ug, tg, n, cg = lts.run(B, dev(U), dev(w.dx), dev(w.nbr.astype(np.int32)), 8 * q,
                            dt_fixed=dev(dtf), dt_quantum=q, check_every=1)
    assert B.check() == 0
    assert n == ns == 8 and np.array_equal(host(cg), cnt) and np.array_equal(host(tg), to)
    err = rel_err_fields(L, host(Ug), Uo)
    log(f"    {ns} steps, updates per patch {cnt.min()}..{cnt.max()}: rel err {err.max():.2e}")
    assert err.max() <= 1e-12 * cnt.max(), err


def test_fp32_run_with_fixed_steps_against_fp64_oracle():
    """The same fixed-step schedule in FP32 (times and steps stay FP64): same updates per
    patch, states within the FP32 full-run bar of the FP64 oracle."""
    import oracle
    import torch
    from paper_2508_09568_amd import lts
    log("[gpu] lts run fp32 vs fp64 oracle, fixed per-patch steps")
    w, U = _ot()
    L = w.layout
    U = U.astype(np.float32).astype(np.float64)
    prm = oracle.Params(gamma=w.gamma)
    dtf = 1e-3 * 2.0 ** -(np.arange(L.P) % 3)
    t_end = 4e-3
    Uo, to, cnt, ns = oracle.lts_run(U, L.dims, L.g, w.dx, w.nbr, prm, t_end=t_end, dt_fixed=dtf)
    B = make_bunch(L, w.gamma, precision=4)
    Ug, tg, n, cg = lts.run(B, dev(U).to(torch.float32), dev(w.dx), dev(w.nbr.astype(np.int32)),
                            t_end, dt_fixed=dev(dtf), check_every=1)
    assert B.check() == 0
    assert n == ns and np.array_equal(host(cg), cnt) and np.array_equal(host(tg), to)
    G = host(Ug).astype(np.float64)
    num = np.zeros(8)
    den = np.zeros(8)
    for p in range(L.P):
        a, b = L.interior(G, p).reshape(8, -1), L.interior(Uo, p).reshape(8, -1)
        num += np.abs(a - b).sum(axis=1)
        den += np.abs(b).sum(axis=1)
    err = num / np.maximum(den, 1e-300)
    log(f"    FP32 L1 rel err per field: {err}")
    assert err.max() <= 1e-5, err


def _turb3d(case):
    import oracle
    if case == "periodic":
        w = W.turbulence(N=64, patch=16)                 # 4^3 periodic patches of 16^3
    else:
        w = W.turbulence(N=64, patch=16, grid=(2, 2, 2))  # corner block: outflow faces
    U = w.U.numpy().copy()
    oracle.fill_guards(U, w.layout.dims, w.layout.g, w.nbr)
    return w, U


@pytest.mark.parametrize("case", ["periodic", "outflow_corner"])
@pytest.mark.parametrize("sched", ["fixed", "levels"])
def test_3d_runs_match_oracle_driver(case, sched):
    """3D patches: readiness over all 26 neighbours, edge and corner guards interpolated from
    diagonal owners, and (corner block) outflow guards whose owner is the patch itself.
    Power-of-two fixed steps per patch (1, 1/2, 1/4 of a quantum), or each patch's own CFL
    step halved per patch class and rounded down to quantum x 2^k: exact time sums, so the
    schedule is the oracle's step for step and the states agree to rounding."""
    import oracle
    from paper_2508_09568_amd import lts
    log(f"[gpu] lts 3D run vs oracle, case {case}, schedule {sched}")
    w, U = _turb3d(case)
    L = w.layout
    prm = oracle.Params(gamma=w.gamma, cfl=w.cfl)
    own = oracle.cfl_many(U, L.dims, L.g, w.dx, prm)
    if sched == "fixed":
        q = 2.0 ** np.floor(np.log2(float(own.min())))
        dtf, quantum, t_end = q * 2.0 ** -(np.arange(L.P) % 3), 0.0, 4 * q
    else:
        dtf = own * 2.0 ** -(np.arange(L.P) % 3)
        quantum = 2.0 ** np.floor(np.log2(float(dtf.min())))
        t_end = 8 * quantum
    Uo, to, cnt, ns = oracle.lts_run(U, L.dims, L.g, w.dx, w.nbr, prm, t_end=t_end,
                                     dt_fixed=dtf, dt_quantum=quantum)
    B = make_bunch(L, w.gamma)
    Ug, tg, n, cg = lts.run(B, dev(U), dev(w.dx), dev(w.nbr.astype(np.int32)), t_end,
                            dt_fixed=dev(dtf), dt_quantum=quantum, check_every=1)
    assert B.check() == 0
    assert n == ns and np.array_equal(host(cg), cnt) and np.array_equal(host(tg), to)
    assert cnt.min() < cnt.max()                         # patches at different times
    err = rel_err_fields(L, host(Ug), Uo)
    log(f"    {ns} steps, updates per patch {cnt.min()}..{cnt.max()}: rel err {err.max():.2e}")
    assert err.max() <= 1e-12 * cnt.max(), err


@pytest.mark.parametrize("case", ["periodic", "outflow_corner"])
def test_3d_run_with_own_cfl_steps_matches_oracle_driver(case):
    """Each patch at its own CFL step on an input without symmetry (the seeded 3D turbulence):
    after the first step no two patch times tie, so the readiness rule orders the patches the
    same way on both sides, even though each side takes the steps from its own time-step rule
    (equal to ~1e-13).  The schedule is then the oracle's step for step (steps, updates per
    patch, final times), and the states agree to rounding."""
    import oracle
    from paper_2508_09568_amd import lts
    log(f"[gpu] lts 3D run vs oracle, own CFL steps, case {case}")
    w, U = _turb3d(case)
    L = w.layout
    prm = oracle.Params(gamma=w.gamma, cfl=w.cfl)
    own = oracle.cfl_many(U, L.dims, L.g, w.dx, prm)
    t_end = 2.5 * float(own.min())
    Uo, to, cnt, ns = oracle.lts_run(U, L.dims, L.g, w.dx, w.nbr, prm, t_end=t_end)
    B = make_bunch(L, w.gamma, cfl=w.cfl)
    Ug, tg, n, cg = lts.run(B, dev(U), dev(w.dx), dev(w.nbr.astype(np.int32)), t_end,
                            check_every=1)
    assert B.check() == 0
    assert n == ns and np.array_equal(host(cg), cnt) and np.array_equal(host(tg), to)
    assert np.all(to == t_end) and cnt.min() < cnt.max()
    err = rel_err_fields(L, host(Ug), Uo)
    log(f"    {ns} steps, updates per patch {cnt.min()}..{cnt.max()}: rel err {err.max():.2e}")
    assert err.max() <= 1e-12 * cnt.max(), err


def test_in_place_local_steps_agree_bitwise_across_solver_forms():
    """The update of a local step runs in place and its solver tiles write the previous slice
    (k_solve_keep): one-phase, two-phase and faces-after-edge-pass tiles and the edge-line pass
    give the same bits over a whole own-CFL run (3D periodic turbulence), as the out-of-place
    update does."""
    import torch

    import oracle
    from paper_2508_09568_amd import lts
    log("[gpu] lts in place: solver forms 0-3 over one run")
    w, U = _turb3d("periodic")
    L = w.layout
    prm = oracle.Params(gamma=w.gamma, cfl=w.cfl)
    t_end = 3.0 * float(oracle.cfl_many(U, L.dims, L.g, w.dx, prm).min())
    Ud, dxd, nbd = dev(U), dev(w.dx), dev(w.nbr.astype(np.int32))
    runs = []
    for form in range(4):
        B = make_bunch(L, w.gamma, cfl=w.cfl)
        B.set_solver_split(form)
        Ug, tg, n, cg = lts.run(B, Ud, dxd, nbd, t_end, check_every=1)
        assert B.check() == 0
        runs.append((Ug, tg, cg, n))
    log(f"    {runs[0][3]} steps, updates per patch {int(runs[0][2].min())}..{int(runs[0][2].max())}")
    for Ug, tg, cg, n in runs[1:]:
        assert n == runs[0][3]
        assert torch.equal(tg, runs[0][1]) and torch.equal(cg, runs[0][2])
        assert torch.equal(Ug, runs[0][0])


def test_3d_fp32_run_against_fp64_oracle():
    import oracle
    import torch
    from paper_2508_09568_amd import lts
    log("[gpu] lts 3D fp32 run vs fp64 oracle, periodic, fixed steps")
    w, U = _turb3d("periodic")
    L = w.layout
    U = U.astype(np.float32).astype(np.float64)
    prm = oracle.Params(gamma=w.gamma, cfl=w.cfl)
    own = oracle.cfl_many(U, L.dims, L.g, w.dx, prm)
    q = 2.0 ** np.floor(np.log2(float(own.min())))
    dtf = q * 2.0 ** -(np.arange(L.P) % 3)
    Uo, to, cnt, ns = oracle.lts_run(U, L.dims, L.g, w.dx, w.nbr, prm, t_end=4 * q, dt_fixed=dtf)
    B = make_bunch(L, w.gamma, precision=4)
    Ug, tg, n, cg = lts.run(B, dev(U).to(torch.float32), dev(w.dx), dev(w.nbr.astype(np.int32)),
                            4 * q, dt_fixed=dev(dtf), check_every=1)
    assert B.check() == 0
    assert n == ns and np.array_equal(host(cg), cnt) and np.array_equal(host(tg), to)
    from gpu_util import l1_rel_fields
    l1 = l1_rel_fields(L, host(Ug), Uo)
    log(f"    FP32 L1 rel err per field: {l1}")
    assert l1.max() <= 1e-5, l1


def test_bad_given_step_stops_the_patch_and_is_reported():
    """A ready patch whose given step is NaN, zero or negative does not advance (its state
    and time stay, its step is 0) and the device status reports an invalid argument; the
    other ready patches advance as usual."""
    import torch

    from paper_2508_09568_amd.binding import MHD_EINVAL
    log("[gpu] lts step with NaN / zero / negative given steps")
    w, U = _ot()
    L = w.layout
    B = make_bunch(L, w.gamma)
    dtf = np.full(L.P, 1e-4)
    dtf[[1, 5, 9]] = [np.nan, 0.0, -1e-4]
    Uc, Un, Up = dev(U), dev(np.zeros_like(U)), dev(U)
    t, tp, dt = (torch.zeros(L.P, dtype=torch.float64, device="cuda") for _ in range(3))
    B.lts_step(Uc, Un, Up, t, tp, dt, dev(w.dx), dev(w.nbr.astype(np.int32)), 1.0,
               dt_fixed=dev(dtf))
    assert B.check() == MHD_EINVAL
    assert B.check() == 0
    th, dth, got = host(t), host(dt), host(Uc)
    bad = np.zeros(L.P, dtype=bool)
    bad[[1, 5, 9]] = True
    assert np.all(dth[bad] == 0.0) and np.all(th[bad] == 0.0)
    assert np.all(dth[~bad] == 1e-4) and np.all(th[~bad] == 1e-4)
    for p in np.nonzero(bad)[0]:
        assert np.array_equal(L.interior(got, p), L.interior(U, p))


@pytest.mark.parametrize("case,form", [("periodic", 0), ("outflow_corner", 0), ("periodic", 3)])
def test_compacted_captured_and_chunked_runs_agree_bitwise(case, form):
    """The same local-time-stepping run (each patch at its own CFL step) three ways: one
    chunk, so every step compacts its launch tables to the ready patches (eager calls); the
    same with the steps captured in HIP graphs; and a bunch processed in several scratch
    chunks, whose steps launch over every patch.  All give the same bits and times (solver
    form 0, and form 3, whose edge-line table is compacted as well)."""
    import torch
    from paper_2508_09568_amd import lts
    log(f"[gpu] lts compacted / captured / chunked, case {case}, solver form {form}")
    w, U = _turb3d(case)
    L = w.layout
    import oracle
    prm = oracle.Params(gamma=w.gamma, cfl=w.cfl)
    own = oracle.cfl_many(U, L.dims, L.g, w.dx, prm)
    t_end = 6 * float(own.min())
    Ud, dxd, nbd = dev(U), dev(w.dx), dev(w.nbr.astype(np.int32))
    B1 = make_bunch(L, w.gamma)
    B1.set_solver_split(form)
    Ua, ta, na, ca = lts.run(B1, Ud, dxd, nbd, t_end, check_every=1)
    assert B1.check() == 0
    Ug, tg, ng = lts.run_graph(B1, Ud, dxd, nbd, t_end, steps_per_graph=4)
    assert B1.check() == 0
    per = int(8 * np.prod(L.dims[0] + 2 * L.g)) * 8 * 11   # scratch of about one patch
    Bc = make_bunch(L, w.gamma, max_scratch_bytes=2 * per)
    Uc, tc, nc, cc = lts.run(Bc, Ud, dxd, nbd, t_end, check_every=1)
    assert Bc.check() == 0
    log(f"    {na} steps, updates per patch {int(ca.min())}..{int(ca.max())}; graph launched {ng}")
    assert int(ca.min()) < int(ca.max())
    assert torch.equal(ta, tg) and torch.equal(ta, tc) and torch.equal(ca, cc) and na == nc
    assert torch.equal(Ua, Ug) and torch.equal(Ua, Uc)
