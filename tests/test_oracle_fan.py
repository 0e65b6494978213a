"""Pins of the oracle's HLLD wave fan, time-step rule and edge-EMF solver that a plausible
slip in any of them fails.

* Every intermediate HLLD state satisfies the conservation-law jump conditions
  (Rankine-Hugoniot) across the wave that bounds it, for all 8 components of the paper's
  flux vector (eq:MHD_vector): a wrong weight, sign or energy term in the single-star or
  double-star states breaks one of them.  The HLLD states are defined by exactly these
  conditions (Miyoshi & Kusano 2005, the solver §2.1 "HLLD Solver" / Fig. 1 refers to).
* The flux is continuous where the contact speed changes sign (double-star regions left
  and right of it), and an isolated rotational discontinuity is resolved exactly.
* The time step of a uniform state and of a two-state patch equals the rule
  dt = C / sum_d (|u_d| + c_f,d) / dx_d computed here from the textbook fast speed.
* The four-state edge EMF with data varying along the second transverse direction only
  reduces to the 1D HLL flux of that direction (§2.1 "Constrained transport and
  2D-extension", Fig. 3)."""
import math

import numpy as np
import pytest

import refmath as rm

GAM = 5.0 / 3.0


def _state(rng, bn):
    return np.array([rng.uniform(0.1, 3), rng.standard_normal(), rng.standard_normal(),
                     rng.standard_normal(), rng.uniform(0.05, 3), bn, rng.standard_normal(),
                     rng.standard_normal()])


def _cons(W):
    """Face-frame primitive (rho, u_n, u_t1, u_t2, p, B_n, B_t1, B_t2) -> conserved."""
    return rm.prim_to_cons(W, GAM)


def _degenerate(W, S, SM, bn, tol=1e-4):
    r, u = W[0], W[1]
    dd = r * (S - u) * (S - SM) - bn * bn
    return abs(dd) <= tol * (r * (S - u) ** 2 + bn * bn)


def test_hlld_states_satisfy_jump_conditions_across_every_wave(ora):
    """F(U_{k+1}) - F(U_k) = S_k (U_{k+1} - U_k) for the five waves S_L, S*_L, S_M, S*_R,
    S_R and all eight components, on 10^4 random pairs with B_n != 0 (the intermediate
    states carry the fan's total pressure); and the returned flux is the physical flux of
    the state of the region that contains the face."""
    rng = np.random.default_rng(11)
    prm = ora.Params(gamma=GAM)
    worst, worst_sel, n = 0.0, 0.0, 0
    regions = set()
    while n < 10000:
        bn = rng.choice([-1, 1]) * rng.uniform(0.05, 2.0)
        L, R = _state(rng, bn), _state(rng, bn)
        F, reg, sp, st = ora.hlld_fan(L, R, prm)
        if _degenerate(L, sp[0], sp[2], bn) or _degenerate(R, sp[4], sp[2], bn):
            continue
        n += 1
        regions.add(reg)
        states = [_cons(L), st[0], st[1], st[2], st[3], _cons(R)]
        # outer states: total pressure from the energy relation; intermediate states: the
        # fan's own (constant across it)
        fl = [rm.face_flux8(U, GAM, None if k in (0, 5) else sp[5])
              for k, U in enumerate(states)]
        for k in range(5):
            lhs = fl[k + 1] - fl[k]
            rhs = sp[k] * (states[k + 1] - states[k])
            scale = (np.abs(fl[k]).max() + np.abs(fl[k + 1]).max() +
                     abs(sp[k]) * (np.abs(states[k]).max() + np.abs(states[k + 1]).max()))
            worst = max(worst, np.abs(lhs - rhs).max() / scale)
        sel = fl[reg][:5]
        worst_sel = max(worst_sel, np.abs(F - sel).max() / (np.abs(sel).max() + 1.0))
    assert worst <= 1e-12, worst
    assert worst_sel <= 1e-12, worst_sel
    assert regions == {0, 1, 2, 3, 4, 5}


def test_hlld_flux_continuous_where_contact_speed_changes_sign(ora):
    """Moving both states by a common normal velocity moves every wave speed by the same
    amount; just left and just right of S_M = 0 the face lies in the left and right
    double-star regions and the two fluxes differ by O(shift), not O(1)."""
    rng = np.random.default_rng(12)
    prm = ora.Params(gamma=GAM)
    worst = 0.0
    for _ in range(3000):
        bn = rng.choice([-1, 1]) * rng.uniform(0.05, 2.0)
        L, R = _state(rng, bn), _state(rng, bn)
        if abs(L[0] - R[0]) < 0.2:
            R[0] += 0.5        # unequal densities: the double-star weights differ
        _, _, sp, _ = ora.hlld_fan(L, R, prm)
        h = 1e-9 * (abs(sp[2]) + 1.0)
        out = []
        for c in (-sp[2] - h, -sp[2] + h):
            Ls, Rs = L.copy(), R.copy()
            Ls[1] += c
            Rs[1] += c
            F, reg, sp2, _ = ora.hlld_fan(Ls, Rs, prm)
            out.append((F, reg))
        (Fm, rm_), (Fp, rp) = out
        assert rm_ == 3 and rp == 2, (rm_, rp)   # S_M < 0: right of contact; > 0: left
        worst = max(worst, np.abs(Fp - Fm).max() / (np.abs(Fp).max() + 1.0))
    assert worst <= 1e-6, worst


@pytest.mark.parametrize("sign_bn", [1.0, -1.0])
@pytest.mark.parametrize("going", ["left", "right"])
def test_hlld_resolves_isolated_rotational_discontinuity(ora, sign_bn, going):
    """Equal rho, p, u_n and |B_t| on both sides, B_t rotated, with the tangential velocity
    jump of an Alfven wave (dv_t = +-sign(B_n) dB_t / sqrt(rho)).  A left-going wave with
    0 <= u_n < |B_n|/sqrt(rho) leaves the face in the left double-star region, whose state
    must be U_R exactly; a right-going one with -|B_n|/sqrt(rho) < u_n < 0 gives U_L."""
    rng = np.random.default_rng(13 if going == "left" else 14)
    prm = ora.Params(gamma=GAM)
    for _ in range(300):
        rho = rng.uniform(0.2, 3.0)
        p = rng.uniform(0.1, 2.0)
        bn = sign_bn * rng.uniform(0.3, 2.0)
        ca = abs(bn) / math.sqrt(rho)
        bt = rng.uniform(0.2, 2.0)
        th0, th1 = rng.uniform(0, 2 * math.pi, 2)
        BL = bt * np.array([math.cos(th0), math.sin(th0)])
        BR = bt * np.array([math.cos(th1), math.sin(th1)])
        vL = rng.standard_normal(2)
        sgn = 1.0 if bn > 0 else -1.0
        if going == "left":
            un = rng.uniform(0.0, 0.9) * ca
            vR = vL + sgn * (BR - BL) / math.sqrt(rho)
        else:
            un = -rng.uniform(0.05, 0.9) * ca
            vR = vL - sgn * (BR - BL) / math.sqrt(rho)
        L = np.array([rho, un, *vL, p, bn, *BL])
        R = np.array([rho, un, *vR, p, bn, *BR])
        F, reg = ora.hlld(L, R, prm)
        if going == "left":
            assert reg == 2
            ref = rm.face_flux8(_cons(R), GAM)[:5]
        else:
            assert reg == 3
            ref = rm.face_flux8(_cons(L), GAM)[:5]
        np.testing.assert_allclose(F, ref, rtol=0, atol=1e-13 * (np.abs(ref).max() + 1.0))


# ---------------------------------------------------------------------------- time step

def _hand_dt(q, dx, act, cfl=0.4):
    """C / sum over active d of (|u_d| + c_f,d)/dx_d, c_f,d from the textbook closed form
    with B_d as the normal field."""
    rho, u, p, B = q[0], q[1:4], q[4], q[5:8]
    s = 0.0
    for d in range(3):
        if not act[d]:
            continue
        cf = rm.cfast_textbook(rho, p, B[d], B[(d + 1) % 3], B[(d + 2) % 3], GAM)
        s += (abs(u[d]) + cf) / dx[d]
    return cfl / s


def _uniform_patch(n, g, q):
    N = [m + 2 * g if m > 1 else 1 for m in n]
    U = np.empty((8, N[2], N[1], N[0]))
    Uc = rm.prim_to_cons(np.asarray(q, float), GAM)
    for m in range(8):
        U[m] = Uc[m]
    return U


@pytest.mark.parametrize("n,act", [((5, 6, 7), (1, 1, 1)), ((8, 6, 1), (1, 1, 0)),
                                   ((9, 1, 1), (1, 0, 0))])
def test_cfl_of_uniform_state_by_hand(ora, n, act):
    """Oblique velocity and field, three different spacings: every active direction
    contributes its own (|u_d| + c_f,d)/dx_d to one sum (a max instead of the sum, a
    wrong normal field or a wrong C fails).  Collapsed directions contribute nothing."""
    g = 3
    prm = ora.Params(gamma=GAM, cfl=0.4)
    dx = np.array([0.1, 0.07, 0.13])
    rng = np.random.default_rng(15)
    for _ in range(20):
        q = np.array([rng.uniform(0.3, 2), *rng.standard_normal(3), rng.uniform(0.2, 2),
                      *rng.standard_normal(3)])
        U = _uniform_patch(n, g, q)
        got = ora.cfl_many(U.ravel(), np.array([n], np.int32), g, dx[None, :], prm)[0]
        ref = _hand_dt(q, dx, act)
        assert got == pytest.approx(ref, rel=1e-13)
        # the fast speed's closed form agrees with the Jacobian's extreme eigenvalue
        qr = np.array([q[0], q[1], q[2], q[3], q[4], q[5], q[6], q[7]])
        lam, _ = rm.wave_eigensystem(qr, GAM)
        assert lam.max() - q[1] == pytest.approx(
            rm.cfast_textbook(q[0], q[4], q[5], q[6], q[7], GAM), rel=1e-9)


def test_cfl_minimum_picks_the_fastest_cell(ora):
    """A patch at rest except one interior cell (its own velocity and pressure, field
    uniform): the step is that cell's by hand, wherever the cell sits; a cell in the
    guards does not count."""
    g = 3
    n = (6, 5, 4)
    prm = ora.Params(gamma=GAM, cfl=0.4)
    dx = np.array([0.05, 0.04, 0.06])
    q0 = np.array([1.0, 0.1, -0.2, 0.05, 0.6, 0.3, -0.2, 0.4])
    q1 = np.array([0.7, -1.3, 0.9, 0.4, 2.5, 0.3, -0.2, 0.4])
    rng = np.random.default_rng(16)
    for _ in range(10):
        U = _uniform_patch(n, g, q0)
        i, j, k = (g + rng.integers(0, n[0]), g + rng.integers(0, n[1]),
                   g + rng.integers(0, n[2]))
        U[:, k, j, i] = rm.prim_to_cons(q1, GAM)
        got = ora.cfl_many(U.ravel(), np.array([n], np.int32), g, dx[None, :], prm)[0]
        assert got == pytest.approx(min(_hand_dt(q0, dx, (1, 1, 1)),
                                        _hand_dt(q1, dx, (1, 1, 1))), rel=1e-13)
        # the same fast state in a guard cell is ignored
        U = _uniform_patch(n, g, q0)
        U[:, 1, 2, 0] = rm.prim_to_cons(q1, GAM)
        got = ora.cfl_many(U.ravel(), np.array([n], np.int32), g, dx[None, :], prm)[0]
        assert got == pytest.approx(_hand_dt(q0, dx, (1, 1, 1)), rel=1e-13)


# ------------------------------------------------------------------------ edge EMF

def test_uct_reduces_to_1d_hll_along_second_direction(ora):
    """With identical states across the first transverse direction (SW = SE = S and
    NW = NE = N), EMF_z is minus the 1D HLL flux along y of B_x (y-flux of Bx = v Bx - u By
    = -EMF_z in eq:MHD_vector), with outer speeds from the fast speed along y (normal field
    B_y, continuous across the edge)."""
    rng = np.random.default_rng(17)
    prm = ora.Params(gamma=GAM)
    worst = 0.0
    for _ in range(3000):
        S = np.array([rng.uniform(0.1, 3), *rng.standard_normal(3), rng.uniform(0.05, 3),
                      *rng.standard_normal(3)])
        N = np.array([rng.uniform(0.1, 3), *rng.standard_normal(3), rng.uniform(0.05, 3),
                      *rng.standard_normal(3)])
        N[6] = S[6]
        ez = ora.uct([S, S, N, N], prm)        # SW, SE, NW, NE
        cs = rm.cfast_textbook(S[0], S[4], S[6], S[7], S[5], GAM)
        cn = rm.cfast_textbook(N[0], N[4], N[6], N[7], N[5], GAM)
        ap = max(0.0, S[2] + cs, N[2] + cn)
        am = max(0.0, cs - S[2], cn - N[2])
        FS = S[2] * S[5] - S[1] * S[6]
        FN = N[2] * N[5] - N[1] * N[6]
        ref = -(ap * FS + am * FN - ap * am * (N[5] - S[5])) / (ap + am)
        worst = max(worst, abs(ez - ref) / (abs(ref) + 1.0))
    assert worst <= 1e-13, worst
