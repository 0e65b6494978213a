"""Independent reference mathematics used to pin the oracle (numpy only).

Nothing here is shared with the oracle or the GPU library:
  * exact Riemann solver for the Euler equations (Toro, ch. 4: pressure function,
    Newton iteration for p*, self-similar sampling),
  * HLLC flux (Toro, ch. 10) for the B = 0 reduction of HLLD,
  * the conservative ideal-MHD flux vector of the paper's eq:MHD_vector written for an
    arbitrary direction, with complex-step Jacobians,
  * eigen-decomposition of the 1D primitive system for linear-wave initial data,
  * the one-dimensional HLL flux of a transverse field component.
"""
from __future__ import annotations

import math

import numpy as np


# ------------------------------------------------------------------ exact Riemann solver

def _pressure_fn(p, rk, pk, gamma):
    ak = math.sqrt(gamma * pk / rk)
    if p > pk:   # shock branch
        A = 2.0 / ((gamma + 1.0) * rk)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        f = (p - pk) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - (p - pk) / (2.0 * (B + p)))
    else:        # rarefaction branch
        f = 2.0 * ak / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
        df = 1.0 / (rk * ak) * (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr, gamma):
    """(p*, u*) of the Euler Riemann problem by Newton iteration on the pressure
    function (Toro §4.3)."""
    p = max(1e-12, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) *
            (math.sqrt(gamma * pl / rl) + math.sqrt(gamma * pr / rr)))
    for _ in range(200):
        fl, dl = _pressure_fn(p, rl, pl, gamma)
        fr, dr = _pressure_fn(p, rr, pr, gamma)
        pn = p - (fl + fr + ur - ul) / (dl + dr)
        pn = max(pn, 1e-14)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _pressure_fn(p, rl, pl, gamma)
    fr, _ = _pressure_fn(p, rr, pr, gamma)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def exact_riemann(rl, ul, pl, rr, ur, pr, gamma, x, t, x0=0.5):
    """Exact (rho, u, p) at positions x, time t (Toro §4.5 sampling)."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, gamma)
    al, ar = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    out = np.zeros((3, len(x)))
    for n, xi in enumerate(np.asarray(x, dtype=float)):
        s = (xi - x0) / t
        if s <= us:   # left of contact
            if ps > pl:   # left shock
                sl = ul - al * math.sqrt((gamma + 1) / (2 * gamma) * ps / pl + (gamma - 1) / (2 * gamma))
                if s <= sl:
                    w = (rl, ul, pl)
                else:
                    w = (rl * (ps / pl + g1) / (g1 * ps / pl + 1.0), us, ps)
            else:          # left rarefaction
                shl = ul - al
                asl = al * (ps / pl) ** ((gamma - 1) / (2 * gamma))
                stl = us - asl
                if s <= shl:
                    w = (rl, ul, pl)
                elif s >= stl:
                    w = (rl * (ps / pl) ** (1.0 / gamma), us, ps)
                else:
                    c = 2.0 / (gamma + 1) + g1 / al * (ul - s)
                    w = (rl * c ** (2.0 / (gamma - 1)),
                         2.0 / (gamma + 1) * (al + (gamma - 1) / 2 * ul + s),
                         pl * c ** (2 * gamma / (gamma - 1)))
        else:         # right of contact
            if ps > pr:
                sr = ur + ar * math.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
                if s >= sr:
                    w = (rr, ur, pr)
                else:
                    w = (rr * (ps / pr + g1) / (g1 * ps / pr + 1.0), us, ps)
            else:
                shr = ur + ar
                asr = ar * (ps / pr) ** ((gamma - 1) / (2 * gamma))
                str_ = us + asr
                if s >= shr:
                    w = (rr, ur, pr)
                elif s <= str_:
                    w = (rr * (ps / pr) ** (1.0 / gamma), us, ps)
                else:
                    c = 2.0 / (gamma + 1) - g1 / ar * (ur - s)
                    w = (rr * c ** (2.0 / (gamma - 1)),
                         2.0 / (gamma + 1) * (-ar + (gamma - 1) / 2 * ur + s),
                         pr * c ** (2 * gamma / (gamma - 1)))
        out[:, n] = w
    return out


def sod_wave_positions(gamma=1.4, t=0.2, x0=0.5):
    rl, ul, pl, rr, ur, pr = 1.0, 0.0, 1.0, 0.125, 0.0, 0.1
    ps, us = star_state(rl, ul, pl, rr, ur, pr, gamma)
    al = math.sqrt(gamma * pl / rl)
    ar = math.sqrt(gamma * pr / rr)
    asl = al * (ps / pl) ** ((gamma - 1) / (2 * gamma))
    sr = ur + ar * math.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
    g1 = (gamma - 1) / (gamma + 1)
    return {
        "p_star": ps, "u_star": us,
        "rho_star_L": rl * (ps / pl) ** (1.0 / gamma),
        "rho_star_R": rr * (ps / pr + g1) / (g1 * ps / pr + 1.0),
        "shock_speed": sr,
        "fan_head": x0 + (ul - al) * t, "fan_tail": x0 + (us - asl) * t,
        "contact": x0 + us * t, "shock": x0 + sr * t,
    }


# ------------------------------------------------------------------------------- HLLC

def hllc(L, R, gamma, SL, SR):
    """HLLC flux (Toro §10.4) for the Euler equations with given outer speeds.
    States (rho, u, v, w, p); returns (rho, m_n, m_t1, m_t2, E) fluxes."""
    rl, ul, vl, wl, pl = L
    rr, ur, vr, wr, pr = R
    El = pl / (gamma - 1) + 0.5 * rl * (ul * ul + vl * vl + wl * wl)
    Er = pr / (gamma - 1) + 0.5 * rr * (ur * ur + vr * vr + wr * wr)
    ss = (pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur)) / (rl * (SL - ul) - rr * (SR - ur))

    def flux(r, u, v, w, p, E):
        return np.array([r * u, r * u * u + p, r * u * v, r * u * w, u * (E + p)])

    def ustar(r, u, v, w, p, E, S):
        f = r * (S - u) / (S - ss)
        return f * np.array([1.0, ss, v, w, E / r + (ss - u) * (ss + p / (r * (S - u)))])

    FL, FR = flux(rl, ul, vl, wl, pl, El), flux(rr, ur, vr, wr, pr, Er)
    if SL >= 0:
        return FL
    if SR <= 0:
        return FR
    UL = np.array([rl, rl * ul, rl * vl, rl * wl, El])
    UR = np.array([rr, rr * ur, rr * vr, rr * wr, Er])
    if ss >= 0:
        return FL + SL * (ustar(rl, ul, vl, wl, pl, El, SL) - UL)
    return FR + SR * (ustar(rr, ur, vr, wr, pr, Er, SR) - UR)


# ----------------------------------------------------------- MHD flux vector & Jacobians

def mhd_flux(U, d, gamma):
    """Flux of the conservative ideal-MHD system along direction d for the cell-centred
    state U = (rho, rho u, rho v, rho w, E, Bx, By, Bz): the paper's eq:MHD_vector with
    x replaced by d (components rotate with the axis).  Works on complex input."""
    rho = U[0]
    u = U[1:4] / rho
    E = U[4]
    B = U[5:8]
    b2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2]
    pg = (gamma - 1.0) * (E - 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) - 0.5 * b2)
    pt = pg + 0.5 * b2
    ub = u[0] * B[0] + u[1] * B[1] + u[2] * B[2]
    F = np.zeros(8, dtype=U.dtype)
    F[0] = rho * u[d]
    for i in range(3):
        F[1 + i] = rho * u[i] * u[d] - B[i] * B[d] + (pt if i == d else 0.0)
        F[5 + i] = B[i] * u[d] - B[d] * u[i]
    F[4] = u[d] * (E + pt) - B[d] * ub
    return F


def prim_to_cons(q, gamma):
    rho, u, v, w, p, bx, by, bz = q
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w) + 0.5 * (bx * bx + by * by + bz * bz)
    return np.array([rho, rho * u, rho * v, rho * w, E, bx, by, bz], dtype=np.result_type(q[0], float))


def cons_to_prim(U, gamma):
    rho = U[0]
    u, v, w = U[1] / rho, U[2] / rho, U[3] / rho
    bx, by, bz = U[5], U[6], U[7]
    p = (gamma - 1.0) * (U[4] - 0.5 * rho * (u * u + v * v + w * w) - 0.5 * (bx * bx + by * by + bz * bz))
    return np.array([rho, u, v, w, p, bx, by, bz], dtype=np.result_type(U[0], float))


def complex_step_jacobian(f, x, h=1e-30):
    """df/dx to rounding accuracy by the complex-step method."""
    x = np.asarray(x, dtype=float)
    n = len(x)
    cols = []
    for j in range(n):
        xc = x.astype(complex)
        xc[j] += 1j * h
        cols.append(np.imag(f(xc)) / h)
    return np.stack(cols, axis=1)


def prim_jacobian(q, d, gamma):
    """A_d(q) with dq/dt = -sum_d A_d dq/dx_d for the conservative system:
    (dq/dU)(dF_d/dU)(dU/dq)."""
    U = prim_to_cons(np.asarray(q, float), gamma)
    JF = complex_step_jacobian(lambda V: mhd_flux(V, d, gamma), U)
    M = complex_step_jacobian(lambda r: prim_to_cons(r, gamma), q)
    Minv = complex_step_jacobian(lambda V: cons_to_prim(V, gamma), U)
    return Minv @ JF @ M


def wave_eigensystem(q0, gamma):
    """Eigenvalues and right eigenvectors (primitive variables, Bx row removed) of the
    1D system along x about the state q0, sorted by eigenvalue."""
    A = prim_jacobian(q0, 0, gamma)
    keep = [0, 1, 2, 3, 4, 6, 7]
    A7 = A[np.ix_(keep, keep)]
    lam, R = np.linalg.eig(A7)
    o = np.argsort(lam.real)
    return lam.real[o], R[:, o].real


def hll_transverse_flux(WL, WR, SLm, SRp):
    """One-dimensional HLL flux along x of By, with outer speeds SL <= 0 <= SR given as
    alpha- = -SL, alpha+ = SR.  W = (rho, u, v, w, p, Bx, By, Bz)."""
    FL = WL[6] * WL[1] - WL[5] * WL[2]
    FR = WR[6] * WR[1] - WR[5] * WR[2]
    ap, am = SRp, SLm
    return (ap * FL + am * FR - ap * am * (WR[6] - WL[6])) / (ap + am)


def cfast_textbook(rho, p, bn, bt1, bt2, gamma):
    """Fast magnetosonic speed in its usual closed form,
    c_f^2 = (a^2 + b^2 + sqrt((a^2 + b^2)^2 - 4 a^2 b_n^2)) / 2 with a^2 = gamma p / rho,
    b^2 = |B|^2 / rho, b_n^2 = B_n^2 / rho."""
    a2 = gamma * p / rho
    b2 = (bn * bn + bt1 * bt1 + bt2 * bt2) / rho
    bn2 = bn * bn / rho
    return math.sqrt(0.5 * (a2 + b2 + math.sqrt((a2 + b2) ** 2 - 4.0 * a2 * bn2)))


def face_flux8(U, gamma, pt=None):
    """All 8 components of the physical flux along the face normal (x) of a face-frame
    conserved state U = (rho, m_n, m_t1, m_t2, E, B_n, B_t1, B_t2).  pt: total pressure
    to use instead of the one of the energy relation (intermediate states of an
    approximate Riemann fan carry their own total pressure)."""
    U = np.asarray(U, dtype=float)
    F = mhd_flux(U, 0, gamma)
    if pt is not None:
        rho = U[0]
        u = U[1] / rho
        b2 = U[5] ** 2 + U[6] ** 2 + U[7] ** 2
        pg = (gamma - 1.0) * (U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / rho - 0.5 * b2)
        d = pt - (pg + 0.5 * b2)
        F[1] += d
        F[4] += u * d
    return F
