"""The oracle's derivative tools against finite differences (CPU).

 - branch signatures: the traced update returns the same bits as the plain one, and its
   signature moves exactly when a limiter branch is crossed;
 - extended precision: the long-double update agrees with the FP64 one to FP64 round-off
   and takes the same branches;
 - tests/golden/adjoint_case_fd50.txt: at every stored entry the oracle's dual-number
   derivative of the 20-step misfit equals the extended-precision central difference
   (both ends on one branch) to 1e-6 (relative to max(|fd|, 1% of the largest |fd|)), and
   the stored entries and one recomputed entry
   are what the generator script produces."""
import os
import sys

import numpy as np
import pytest

import mhdtest as mt
from paper_2508_09568_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
FIXTURE = os.path.join(HERE, "golden", "adjoint_case_fd50.txt")


def _sine_1d(n=32, amp=0.1):
    L, U, dx, nbr, _ = mt.linear_wave_1d(n, "fast", amp=amp)
    return L, U, dx, nbr


def test_traced_update_is_bitwise_the_plain_update(ora):
    L, U, dx, nbr = _sine_1d()
    ora.fill_guards(U, L.dims, L.g, nbr)
    prm = ora.Params()
    dt = ora.cfl_many(U, L.dims, L.g, dx, prm)
    a = ora.step_many(U, L.dims, L.g, dt, dx, prm)
    b, sig = ora.step_sig_many(U, L.dims, L.g, dt, dx, prm)
    assert np.array_equal(a, b)
    _, sig2 = ora.step_sig_many(U, L.dims, L.g, dt, dx, prm)
    assert np.array_equal(sig, sig2) and sig.dtype == np.uint64


def test_signature_moves_with_a_limiter_branch_and_only_then(ora):
    """Cell c of a smooth profile: its backward and forward density differences share a
    sign.  Moving rho_c by a small amount keeps every branch; moving it past its right
    neighbour flips the sign of the forward difference (a limiter kink)."""
    L, U, dx, nbr = _sine_1d()
    prm = ora.Params()
    g = L.g
    V = L.view(U, 0)
    c = g + 5
    dm = V[0, 0, 0, c] - V[0, 0, 0, c - 1]
    dp = V[0, 0, 0, c + 1] - V[0, 0, 0, c]
    assert dm * dp > 0
    ora.fill_guards(U, L.dims, L.g, nbr)
    dt = ora.cfl_many(U, L.dims, L.g, dx, prm)
    _, s0 = ora.step_sig_many(U, L.dims, L.g, dt, dx, prm)
    U1 = U.copy()
    L.view(U1, 0)[0, 0, 0, c] += 1e-3 * abs(dp)
    _, s1 = ora.step_sig_many(U1, L.dims, L.g, dt, dx, prm)
    assert np.array_equal(s0, s1)
    U2 = U.copy()
    L.view(U2, 0)[0, 0, 0, c] += 2.0 * dp
    _, s2 = ora.step_sig_many(U2, L.dims, L.g, dt, dx, prm)
    assert not np.array_equal(s0, s2)


def test_extended_precision_update_agrees_with_fp64(ora):
    # noise lifts the exact ties of the symmetric initial data, which rounding would decide
    w = W.orszag_tang(32, 16)
    L = w.layout
    U = w.U.copy()
    M = np.zeros(L.total, dtype=bool)
    for p in range(L.P):
        L.interior(M, p)[:] = True
    U[M] += 1e-4 * np.random.default_rng(11).standard_normal(int(M.sum()))
    ora.fill_guards(U, L.dims, L.g, w.nbr)
    prm = ora.Params(gamma=w.gamma)
    dt = ora.cfl_many(U, L.dims, L.g, w.dx, prm)
    a, sa = ora.step_sig_many(U, L.dims, L.g, dt, w.dx, prm)
    Ul = U.astype(np.longdouble)
    ora.fill_guards_ext(Ul, L.dims, L.g, w.nbr)
    b, sb = ora.step_ext_many(Ul, L.dims, L.g, dt, w.dx, prm)
    assert b.dtype == np.longdouble
    assert np.array_equal(sa, sb)
    d = np.abs(a - b.astype(np.float64)).max() / np.abs(a).max()
    assert 0 < d <= 1e-14


def _fixture():
    dt = None
    for line in open(FIXTURE):
        if line.startswith("# dt "):
            dt = float(line.split()[2])
    return np.loadtxt(FIXTURE, comments="#", ndmin=2), dt


def _gen():
    sys.path.insert(0, os.path.join(HERE, "golden"))
    try:
        import make_adjoint_fd
    finally:
        sys.path.pop(0)
    return make_adjoint_fd


def test_fixture_dual_numbers_agree_with_extended_finite_differences():
    rows, dt = _fixture()
    assert rows.shape == (50, 5)
    jv, fd, h, clean = rows[:, 1], rows[:, 2], rows[:, 3], rows[:, 4]
    assert np.all(clean == 1)
    assert np.all((h > 0) & (h <= 1e-8))
    # an entry whose derivative is far below the others' carries the FD round-off (~1e-12
    # absolute at these steps) at full weight: errors are relative to max(|fd|, 1% of the
    # largest |fd| of the 50)
    rel = np.abs(jv - fd) / np.maximum(np.abs(fd), 1e-2 * np.abs(fd).max())
    assert rel.max() <= 1e-6, rel.max()
    assert np.median(np.abs(jv - fd) / np.abs(fd)) <= 1e-7


def test_fixture_entries_are_the_seeded_selection():
    gen = _gen()
    w, L, prm, dt, U0, tgt, owned, rho, pick = gen.setup()
    rows, fdt = _fixture()
    assert np.array_equal(rows[:, 0].astype(np.int64), pick.astype(np.int64))
    assert fdt == dt


@pytest.mark.slow
def test_fixture_first_entry_recomputes(ora):
    """The stored jvp and fd of the first entry are what the generator computes now."""
    gen = _gen()
    w, L, prm, dt, U0, tgt, owned, rho, pick = gen.setup()
    rows, _ = _fixture()
    dts = np.full(L.P, dt)
    ora.fill_guards(tgt, L.dims, L.g, w.nbr)
    rt = gen.rollout(tgt, w, L, prm, dts)
    j = int(pick[0])
    dj = gen.jvp(j, U0, rt, w, L, prm, dts, rho)
    assert dj == rows[0, 1]
    _, s0 = gen.rollout_ext(U0, w, L, prm, dts)
    fj, h, clean = gen.fd(j, U0, rt.astype(np.longdouble), s0, w, L, prm, dts, rho)
    assert clean == 1 and h == rows[0, 3]
    assert fj == rows[0, 2]
