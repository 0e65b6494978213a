"""Writes adjoint_case_fd50.txt: reference derivatives of the adjoint configuration's
misfit at 50 seeded entries of the initial state, from the oracle only.

Configuration: 64^3 periodic as 2x2x2 patches of 32^3, fast wave (amplitude 1e-3) plus
Gaussian noise (1e-4, seed 5) on the uniform background rho=1, p=0.6, B=(1,0,0); 20 steps
at the fixed dt of the noise-free state (C=0.4); misfit L = 1/2 sum over owned cells of
(rho^20 - rho_target)^2 with the target the same configuration under noise seed 6.
Entries: 50 owned (field, cell) DOFs drawn with numpy default_rng(7).

Per entry two independent derivatives:
  jvp -- forward-mode dual numbers through the FP64 oracle's 20 updates;
  fd  -- central difference (L(x+h e_j) - L(x-h e_j)) / 2h of the oracle's rollout in
         x87 extended precision (64-bit significand), h = 1e-8, the misfit difference
         formed cell-wise as sum (r+ - r-)(r+ + r- - 2 r_t) / 2.  The branch signatures of
         every patch update at x+h and x-h must equal those at x (both ends on the smooth
         branch the derivative belongs to); otherwise h is divided by 4, at most 3 times.
         An entry still crossing a branch is written with clean=0, not dropped.

Run from the repository root:  python tests/golden/make_adjoint_fd.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2508_09568_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_case_fd50.txt")
NSTEPS, H0, NENTRY = 20, 1e-8, 50


def setup():
    w = W.adjoint_case()
    L = w.layout
    prm = oracle.Params(gamma=w.gamma)
    clean = W.adjoint_case(noise=0.0)
    Uc = clean.U.copy()
    oracle.fill_guards(Uc, L.dims, L.g, w.nbr)
    dt = float(oracle.cfl_many(Uc, L.dims, L.g, w.dx, prm).min())
    U0 = w.U.copy()
    oracle.fill_guards(U0, L.dims, L.g, w.nbr)
    tgt = W.adjoint_case(noise_seed=6).U.copy()
    owned = np.zeros(L.total, dtype=bool)
    rho = np.zeros(L.total, dtype=bool)
    for p in range(L.P):
        L.interior(owned, p)[:] = True
        L.interior(rho, p)[0] = True
    rng = np.random.default_rng(7)
    pick = rng.choice(np.nonzero(owned)[0], size=NENTRY, replace=False)
    return w, L, prm, dt, U0, tgt, owned, rho, pick


def rollout(U, w, L, prm, dts):
    U = U.copy()
    for _ in range(NSTEPS):
        oracle.fill_guards(U, L.dims, L.g, w.nbr)
        U = oracle.step_many(U, L.dims, L.g, dts, w.dx, prm)
    return U


def rollout_ext(U, w, L, prm, dts):
    U = U.astype(np.longdouble)
    sigs = []
    for _ in range(NSTEPS):
        oracle.fill_guards_ext(U, L.dims, L.g, w.nbr)
        U, s = oracle.step_ext_many(U, L.dims, L.g, dts, w.dx, prm)
        sigs.append(s)
    return U, np.concatenate(sigs)


def jvp(j, U0, rt, w, L, prm, dts, rho):
    U, v = U0.copy(), np.zeros(L.total)
    v[j] = 1.0
    for _ in range(NSTEPS):
        oracle.fill_guards(U, L.dims, L.g, w.nbr)
        oracle.fill_guards(v, L.dims, L.g, w.nbr)
        U, v = oracle.jvp_many(U, v, L.dims, L.g, dts, w.dx, prm)
    return float(np.sum(((U - rt) * v)[rho]))


def fd(j, U0, rtl, s0, w, L, prm, dts, rho):
    h = H0
    for tries in range(4):
        hl = np.longdouble(h)
        up = U0.astype(np.longdouble)
        um = up.copy()
        up[j] += hl
        um[j] -= hl
        rp, sp = rollout_ext(up, w, L, prm, dts)
        rm, sm = rollout_ext(um, w, L, prm, dts)
        d = float(((rp - rm) * (rp + rm - 2 * rtl))[rho].sum() / (4 * hl))
        clean = np.array_equal(sp, s0) and np.array_equal(sm, s0)
        if clean or tries == 3:
            return d, h, int(clean)
        h /= 4


def main():
    w, L, prm, dt, U0, tgt, owned, rho, pick = setup()
    dts = np.full(L.P, dt)
    oracle.fill_guards(tgt, L.dims, L.g, w.nbr)
    rt = rollout(tgt, w, L, prm, dts)
    rtl = rt.astype(np.longdouble)
    _, s0 = rollout_ext(U0, w, L, prm, dts)
    rows = []
    t0 = time.time()
    for k, j in enumerate(pick):
        j = int(j)
        dj = jvp(j, U0, rt, w, L, prm, dts, rho)
        fj, h, clean = fd(j, U0, rtl, s0, w, L, prm, dts, rho)
        rows.append((j, dj, fj, h, clean))
        print(f"[{k + 1}/{NENTRY}] entry {j}: jvp {dj:.15e} fd {fj:.15e} h {h:.3e} clean {clean} "
              f"rel {abs(dj - fj) / abs(fj):.2e} ({time.time() - t0:.0f} s)", flush=True)
    with open(OUT, "w") as f:
        f.write("# adjoint configuration (64^3, 8 patches of 32^3, 20 steps at fixed dt): dL/dU0 "
                "at 50 owned entries\n")
        f.write("# written by tests/golden/make_adjoint_fd.py from the oracle only\n")
        f.write(f"# dt {dt:.17e}\n")
        f.write("# entry  jvp_fp64_dual  fd_extended  h  clean\n")
        for j, dj, fj, h, clean in rows:
            f.write(f"{j} {dj:.17e} {fj:.17e} {h:.6e} {clean}\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
