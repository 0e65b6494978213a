"""Pins of the oracle's local time stepping (patches advancing at their own time step,
guard zones interpolated in time from the neighbours' two slices): the interpolated guard
fill against the plain fill and against a state that is linear in time, the readiness
rule on a toy neighbour table, and the whole driver against synchronous stepping."""
import numpy as np

from paper_2508_09568_amd import workloads as W


def _ot(ora, patch=16):
    w = W.orszag_tang(64, patch)
    U = w.U.copy()
    ora.fill_guards(U, w.layout.dims, w.layout.g, w.nbr)
    return w, U


def test_one_slice_or_equal_times_is_the_plain_fill(ora):
    w, U = _ot(ora)
    L = w.layout
    rng = np.random.default_rng(1)
    ref = U.copy()
    ora.fill_guards(ref, L.dims, L.g, w.nbr)
    junk = rng.standard_normal(U.shape)              # U_prev must not matter
    # owners with a single slice (t == t_prev): the current value
    t = rng.uniform(0.0, 1.0, L.P)
    a = U.copy()
    a[:] = rng.standard_normal(U.shape)              # guards start as garbage
    for p in range(L.P):
        L.interior(a, p)[...] = L.interior(U, p)
    ora.fill_guards_at(a, junk, t, t.copy(), L.dims, L.g, w.nbr)
    assert np.array_equal(a, ref)
    # every patch at the same time, owners' previous slices earlier: th = 1 exactly
    b = a.copy()
    ora.fill_guards_at(b, junk, np.full(L.P, 0.7), np.full(L.P, 0.2), L.dims, L.g, w.nbr)
    assert np.array_equal(b, ref)


def test_state_linear_in_time_is_reproduced(ora):
    """Owner slices U = A + B t[q] and U_prev = A + B t_prev[q]: a guard cell of p takes its
    owner's A + B t[p] (linear interpolation is exact on a linear history)."""
    w, _ = _ot(ora)
    L = w.layout
    rng = np.random.default_rng(2)
    A = rng.standard_normal(L.total)
    Bv = rng.standard_normal(L.total)
    tp = rng.uniform(0.0, 0.4, L.P)
    t = tp + rng.uniform(0.2, 0.6, L.P)
    per = np.diff(L.base)
    U = A + Bv * np.repeat(t, per)
    Up = A + Bv * np.repeat(tp, per)
    got = U.copy()
    ora.fill_guards_at(got, Up, t, tp, L.dims, L.g, w.nbr)
    Af, Bf = A.copy(), Bv.copy()
    ora.fill_guards(Af, L.dims, L.g, w.nbr)
    ora.fill_guards(Bf, L.dims, L.g, w.nbr)
    want = Af + Bf * np.repeat(t, per)
    guard = np.ones(L.total, dtype=bool)
    for p in range(L.P):
        L.interior(guard, p)[...] = False
    assert np.abs(got - want)[guard].max() <= 1e-14 * np.abs(want).max()
    assert np.array_equal(got[~guard], U[~guard])
    # the masked-out patches keep their guards
    got2 = U.copy()
    mask = np.arange(L.P) % 2
    ora.fill_guards_at(got2, Up, t, tp, L.dims, L.g, w.nbr, mask=mask)
    for p in range(L.P):
        a, b = L.view(got2, p), L.view(got if mask[p] else U, p)
        assert np.array_equal(a, b)


def test_readiness_rule_on_a_row_of_patches(ora):
    # four patches in a periodic row along x
    nbr = W.grid_neighbours((4, 1, 1), (True, True, True))
    t = np.array([0.0, 0.1, 0.1, 0.05])
    ready = ora.lts_ready(t, 1.0, nbr)
    assert ready.tolist() == [True, False, False, False]
    assert ora.lts_ready(np.full(4, 0.3), 1.0, nbr).all()
    assert not ora.lts_ready(np.full(4, 1.0), 1.0, nbr).any()


def test_common_fixed_step_equals_synchronous_stepping_bitwise(ora):
    w, U = _ot(ora)
    L = w.layout
    prm = ora.Params(gamma=w.gamma)
    dt = 2e-3
    Ul, t, cnt, ns = ora.lts_run(U, L.dims, L.g, w.dx, w.nbr, prm, t_end=5 * dt - 1e-12,
                                 dt_fixed=np.full(L.P, dt))
    Us = ora.run(U, L.dims, L.g, w.dx, w.nbr, prm, nsteps=4, dt_fixed=dt)
    assert ns == 5 and np.all(cnt == 5)
    # the first four steps are synchronous; compare after a fifth synchronous step
    Us = ora.step_many(ora.fill_guards(Us, L.dims, L.g, w.nbr), L.dims, L.g,
                       np.full(L.P, 5 * dt - 1e-12 - 4 * dt), w.dx, prm)
    for p in range(L.P):
        assert np.array_equal(L.interior(Ul, p), L.interior(Us, p))


def test_cfl_driven_run_stays_close_to_synchronous_stepping(ora):
    """Own CFL steps per patch with interpolated guards against the global-minimum step:
    both are second-order approximations of the same solution."""
    w, U = _ot(ora)
    L = w.layout
    prm = ora.Params(gamma=w.gamma)
    Ul, t, cnt, ns = ora.lts_run(U, L.dims, L.g, w.dx, w.nbr, prm, t_end=0.02)
    Us = ora.run(U, L.dims, L.g, w.dx, w.nbr, prm, t_end=0.02)
    assert np.all(t == 0.02) and ns > cnt.max()
    num = sum(np.abs(L.interior(Ul, p) - L.interior(Us, p)).sum() for p in range(L.P))
    den = sum(np.abs(L.interior(Us, p)).sum() for p in range(L.P))
    assert num / den < 1e-3, num / den


def test_time_levels_round_steps_to_powers_of_two_of_the_quantum(ora):
    """dt_quantum > 0: every step is dt_quantum x 2^k, at most the patch's own step, so the
    patches advance in lock-step groups (with a power-of-two quantum every time is an exact
    sum); the run ends at t_end close to synchronous stepping."""
    w, U = _ot(ora)
    L = w.layout
    prm = ora.Params(gamma=w.gamma)
    own = ora.cfl_many(U, L.dims, L.g, w.dx, prm)
    q = 2.0 ** np.floor(np.log2(0.7 * float(own.min())))   # a power of two: exact time sums
    dtf = own * np.linspace(1.0, 3.0, L.P)              # spread the steps over a few levels
    Ul, t, cnt, ns = ora.lts_run(U, L.dims, L.g, w.dx, w.nbr, prm, t_end=8 * q, dt_fixed=dtf,
                                 dt_quantum=q)
    _, e = np.frexp(dtf / q)
    lev = np.ldexp(q, e - 1)
    assert np.all(lev <= dtf) and np.all(2 * lev > dtf)
    assert np.all(t == 8 * q)
    assert np.array_equal(cnt, np.ceil(8 * q / lev).astype(np.int64))
    assert ns == 8                                       # the finest level sets the step count
    Us = ora.run(U, L.dims, L.g, w.dx, w.nbr, prm, nsteps=8, dt_fixed=q)
    num = sum(np.abs(L.interior(Ul, p) - L.interior(Us, p)).sum() for p in range(L.P))
    den = sum(np.abs(L.interior(Us, p)).sum() for p in range(L.P))
    assert num / den < 1e-3, num / den
