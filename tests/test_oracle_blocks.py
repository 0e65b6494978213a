"""Pins of the oracle's building blocks against mathematics that does not come from the
oracle: limiter tables, eigenvalues of the paper's flux Jacobian, the B = 0 reduction
of HLLD to HLLC, flux consistency, the 1D reduction of the edge-EMF solver to an HLL
flux, and the predictor's time derivative against the conservative flux vector."""
import math

import numpy as np
import pytest

import refmath as rm

GAM = 5.0 / 3.0


def P(ora, **kw):
    return ora.Params(**kw)


# ------------------------------------------------------------------ limiters (tables)

@pytest.mark.parametrize("dl,dr,mc,mm", [
    (1.0, 3.0, 2.0, 1.0),        # MC: min(2, 6, 2) = 2
    (1.0, 1.5, 1.25, 1.0),       # MC: min(2, 3, 1.25)
    (3.0, 1.0, 2.0, 1.0),
    (-3.0, -1.0, -2.0, -1.0),
    (-1.0, 2.0, 0.0, 0.0),       # opposite signs
    (0.0, 1.0, 0.0, 0.0),        # zero on one side
    (2.0, 2.0, 2.0, 2.0),        # smooth: central difference
    (1e-3, 5.0, 2e-3, 1e-3),
])
def test_limiter_table(ora, dl, dr, mc, mm):
    assert ora.limiter(dl, dr, 0) == pytest.approx(mc, rel=0, abs=1e-15)
    assert ora.limiter(dl, dr, 1) == pytest.approx(mm, rel=0, abs=1e-15)


def test_limiter_symmetry(ora):
    rng = np.random.default_rng(0)
    for _ in range(1000):
        a, b = rng.standard_normal(2)
        for k in (0, 1):
            assert ora.limiter(a, b, k) == ora.limiter(b, a, k)
            assert ora.limiter(-a, -b, k) == -ora.limiter(a, b, k)


# -------------------------------------------------- fast speed vs Jacobian eigenvalues

def test_cfast_is_largest_eigenvalue(ora):
    rng = np.random.default_rng(1)
    for _ in range(200):
        rho = rng.uniform(0.1, 3)
        p = rng.uniform(0.05, 2)
        u = rng.uniform(0.1, 1)
        B = rng.standard_normal(3)
        q = np.array([rho, u, rng.standard_normal(), rng.standard_normal(), p, *B])
        lam, _ = rm.wave_eigensystem(q, GAM)
        cf = ora.cfast(rho, p, B[0], B[1], B[2], GAM)
        assert cf == pytest.approx(lam.max() - u, rel=1e-9)
        assert -cf == pytest.approx(lam.min() - u, rel=1e-9)


def test_cfast_limits(ora):
    # B = 0: sound speed; rho = p = 1, B along n: max(a, b)
    assert ora.cfast(1.0, 1.0, 0, 0, 0, 1.4) == pytest.approx(math.sqrt(1.4), rel=1e-15)
    assert ora.cfast(1.0, 0.6, 2.0, 0, 0, GAM) == pytest.approx(2.0, rel=1e-15)
    # perpendicular field: sqrt(a^2 + b^2)
    assert ora.cfast(2.0, 1.0, 0.0, 1.0, 1.0, GAM) == pytest.approx(
        math.sqrt(GAM * 0.5 + 1.0), rel=1e-14)


# --------------------------------------------------------------------------- HLLD

def _rand_state(rng, B=True):
    s = np.array([rng.uniform(0.1, 3), rng.standard_normal(), rng.standard_normal(),
                  rng.standard_normal(), rng.uniform(0.05, 3), 0.0, 0.0, 0.0])
    if B:
        s[5:8] = rng.standard_normal(3)
    return s


def _flux_face(W, gamma):
    """Physical flux in the face frame from eq:MHD_vector (x direction)."""
    U = rm.prim_to_cons(W, gamma)
    F = rm.mhd_flux(U, 0, gamma)
    return F[[0, 1, 2, 3, 4]]


def test_hlld_consistency(ora):
    """F(U, U) = F(U): the Riemann flux of identical states is the physical flux."""
    rng = np.random.default_rng(2)
    prm = P(ora, gamma=GAM)
    for _ in range(2000):
        W = _rand_state(rng)
        F, _ = ora.hlld(W, W, prm)
        Fe = _flux_face(W, GAM)
        scale = np.abs(Fe).max() + W[0] + W[4] + np.sum(W[5:] ** 2)
        assert np.abs(F - Fe).max() <= 1e-13 * scale


def test_hlld_equals_hllc_for_zero_field(ora):
    """With B = 0 the HLLD fan collapses to three waves: HLLC with the same S_L, S_R."""
    rng = np.random.default_rng(3)
    prm = P(ora, gamma=GAM)
    worst = 0.0
    for _ in range(10000):
        L, R = _rand_state(rng, B=False), _rand_state(rng, B=False)
        F, reg = ora.hlld(L, R, prm)
        al, ar = math.sqrt(GAM * L[4] / L[0]), math.sqrt(GAM * R[4] / R[0])
        SL = min(L[1], R[1]) - max(al, ar)
        SR = max(L[1], R[1]) + max(al, ar)
        Fh = rm.hllc(L[:5], R[:5], GAM, SL, SR)
        scale = np.abs(Fh).max() + 1.0
        worst = max(worst, np.abs(F - Fh).max() / scale)
        assert reg in (0, 1, 4, 5)   # the double-star regions are empty when B_n = 0
    assert worst <= 1e-12


def test_hlld_supersonic_upwinding(ora):
    prm = P(ora, gamma=GAM)
    L = np.array([1.0, 20.0, 0.3, -0.2, 1.0, 0.5, 0.7, -0.1])
    R = np.array([0.5, 19.0, -0.3, 0.2, 0.8, 0.5, -0.7, 0.4])
    F, reg = ora.hlld(L, R, prm)
    assert reg == 0 and np.array_equal(F, _flux_face(L, GAM)) or np.allclose(F, _flux_face(L, GAM), rtol=1e-15, atol=0)
    Lm, Rm = L.copy(), R.copy()
    Lm[1], Rm[1] = -20.0, -19.0
    F, reg = ora.hlld(Lm, Rm, prm)
    assert reg == 5
    np.testing.assert_allclose(F, _flux_face(Rm, GAM), rtol=1e-15)


def test_hlld_isolated_contact_has_no_mass_flux(ora):
    """u = 0, equal pressure and field on both sides: an exact stationary contact."""
    rng = np.random.default_rng(4)
    prm = P(ora, gamma=GAM)
    for _ in range(500):
        B = rng.standard_normal(3)
        p = rng.uniform(0.1, 2)
        L = np.array([rng.uniform(0.1, 3), 0, 0, 0, p, *B])
        R = np.array([rng.uniform(0.1, 3), 0, 0, 0, p, *B])
        F, _ = ora.hlld(L, R, prm)
        pt = p + 0.5 * np.sum(B ** 2)
        assert abs(F[0]) <= 1e-14 * max(L[0], R[0]) * 10
        assert F[1] == pytest.approx(pt - B[0] ** 2, rel=1e-13, abs=1e-14)
        assert abs(F[4]) <= 1e-13 * (pt + 1)


def test_hlld_mirror_symmetry(ora):
    """Reflecting the normal axis swaps L and R and flips normal components."""
    rng = np.random.default_rng(5)
    prm = P(ora, gamma=GAM)
    for _ in range(500):
        L, R = _rand_state(rng), _rand_state(rng)
        R[5] = L[5]
        F, _ = ora.hlld(L, R, prm)
        fl = lambda W: np.array([W[0], -W[1], W[2], W[3], W[4], -W[5], W[6], W[7]])
        G, _ = ora.hlld(fl(R), fl(L), prm)
        # mirrored flux: mass, tangential momentum, energy fluxes change sign; normal
        # momentum flux keeps its sign
        np.testing.assert_allclose(G, [-F[0], F[1], -F[2], -F[3], -F[4]], rtol=1e-12,
                                   atol=1e-12 * (np.abs(F).max() + 1))


# ------------------------------------------------------------------- edge EMF solver

def test_uct_reduces_to_1d_hll(ora):
    """With identical states across the second direction (N = S), the four-state EMF is
    the 1D HLL flux of the transverse field (x-flux of By = EMF_z, eq:MHD_vector)."""
    rng = np.random.default_rng(6)
    prm = P(ora, gamma=GAM)
    for _ in range(2000):
        W, E = _rand_state(rng), _rand_state(rng)
        E[5] = W[5]                       # normal (x) field continuous across the edge
        ez = ora.uct([W, E, W, E], prm)   # SW, SE, NW, NE
        cw = ora.cfast(W[0], W[4], W[5], W[6], W[7], GAM)
        ce = ora.cfast(E[0], E[4], E[5], E[6], E[7], GAM)
        ap = max(0.0, W[1] + cw, E[1] + ce)
        am = max(0.0, cw - W[1], ce - E[1])
        ref = rm.hll_transverse_flux(W, E, am, ap)
        assert ez == pytest.approx(ref, rel=1e-13, abs=1e-14)


def test_uct_uniform_state_is_ideal_emf(ora):
    rng = np.random.default_rng(7)
    prm = P(ora, gamma=GAM)
    for _ in range(200):
        W = _rand_state(rng)
        ez = ora.uct([W, W, W, W], prm)
        assert ez == pytest.approx(W[1] * W[6] - W[2] * W[5], rel=1e-13, abs=1e-14)


# -------------------------------------------- predictor time derivative vs the flux

def test_dqdt_matches_conservative_flux_jacobian(ora):
    """dq/dt of the half-step predictor equals -(dq/dU) sum_d (dF_d/dU)(dU/dq) d_d q for
    the flux vector of eq:MHD_vector, on data with zero divergence of B."""
    rng = np.random.default_rng(8)
    for trial in range(300):
        q = np.array([rng.uniform(0.2, 3), *rng.standard_normal(3), rng.uniform(0.1, 2),
                      *rng.standard_normal(3)])
        act = [1, 1, 1] if trial % 3 == 0 else ([1, 1, 0] if trial % 3 == 1 else [1, 0, 0])
        D = rng.standard_normal((3, 8))
        for d in range(3):
            if not act[d]:
                D[d] = 0.0
        # enforce div B = 0 on the slopes
        nact = sum(act)
        s = sum(D[d, 5 + d] for d in range(3) if act[d])
        for d in range(3):
            if act[d]:
                D[d, 5 + d] -= s / nact
        got = ora.dqdt(q, D, act, GAM)
        ref = np.zeros(8)
        for d in range(3):
            if act[d]:
                ref -= rm.prim_jacobian(q, d, GAM) @ D[d]
        np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())
