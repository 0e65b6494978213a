"""The update with the next step's time step reduced in its own tiles
(mhd_bunch_update_cfl, through the C ABI): the same output as mhd_bunch_update, and a next
time step equal to mhd_bunch_cfl (global minimum) on the output after the guard exchange --
periodic boxes (neighbour faces) and blocks with domain boundaries (copied faces), in every
solver form and tile shape, FP64 and FP32, and a run of several steps."""
import numpy as np
import pytest

from gpu_util import dev, host, log, make_bunch
from paper_2508_09568_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(name):
    import oracle
    if name == "turb_periodic":
        w = W.turbulence(N=64, patch=16)
        U = w.U.numpy().copy()
    elif name == "turb_corner":
        w = W.turbulence(N=64, patch=16, grid=(2, 2, 2))
        U = w.U.numpy().copy()
    elif name == "ot64":
        w = W.orszag_tang(64, 32)
        U = np.ascontiguousarray(w.U, dtype=np.float64).copy()
    else:
        w = W.sod(128, patches=8)
        U = np.ascontiguousarray(w.U, dtype=np.float64).copy()
    oracle.fill_guards(U, w.layout.dims, w.layout.g, w.nbr)
    return w, U


@pytest.mark.parametrize("name", ["turb_periodic", "turb_corner", "ot64", "sod8"])
@pytest.mark.parametrize("precision", [8, 4])
def test_next_time_step_equals_separate_pass(name, precision):
    import torch
    log(f"[gpu] update + next time step case={name} precision={precision}")
    w, U = _case(name)
    L = w.layout
    B = make_bunch(L, w.gamma, precision=precision, cfl=w.cfl)
    dty = torch.float64 if precision == 8 else torch.float32
    Ui = dev(U).to(dty)
    nbr = dev(w.nbr.astype(np.int32))
    dxd = dev(w.dx)
    dt = torch.zeros(L.P, dtype=torch.float64, device="cuda")
    B.cfl(Ui, dxd, dt, global_min=True)
    n = 0
    for fused in range(len(B.predictor_modes())):
        B.set_predictor(fused)
        for split in range(4):
            B.set_solver_split(split)
            for i in range(len(B.tile_configs())):
                B.set_tile(i)
                Ua = torch.zeros_like(Ui)
                Ub = torch.zeros_like(Ui)
                B.update(Ui, Ua, dt, dxd)
                dn = torch.zeros_like(dt)
                B.update_cfl(Ui, Ub, dt, dxd, nbr, dn)
                B.fill_guards(Ua, nbr)
                ref = torch.zeros_like(dt)
                B.cfl(Ua, dxd, ref, global_min=True)
                assert B.check() == 0
                a, b = host(Ua), host(Ub)
                for p in range(L.P):
                    assert np.array_equal(L.interior(a, p), L.interior(b, p)), (fused, split, i, p)
                assert torch.equal(dn, ref), (fused, split, i, float(dn[0]), float(ref[0]))
                n += 1
    log(f"    {n} configurations: same state, next time step {float(ref[0]):.17g} bitwise")


def test_run_with_fused_time_step_matches_separate_passes():
    """Ten steps of guard exchange + update with the fused time step give the bits of the
    steps with the separate time-step pass."""
    import torch
    w, U = _case("turb_periodic")
    L = w.layout
    B = make_bunch(L, w.gamma, cfl=w.cfl)
    nbr = dev(w.nbr.astype(np.int32))
    dxd = dev(w.dx)
    Ua, Ub = dev(U), dev(U)
    dt = torch.zeros(L.P, dtype=torch.float64, device="cuda")
    dt2 = torch.zeros_like(dt)
    B.fill_guards(Ub, nbr)
    B.cfl(Ub, dxd, dt2, global_min=True)
    for _ in range(10):
        B.fill_guards(Ua, nbr)
        B.cfl(Ua, dxd, dt, global_min=True)
        Ua2 = torch.empty_like(Ua)
        B.update(Ua, Ua2, dt, dxd)
        Ua = Ua2
        B.fill_guards(Ub, nbr)
        Ub2 = torch.empty_like(Ub)
        dn = torch.empty_like(dt2)
        B.update_cfl(Ub, Ub2, dt2, dxd, nbr, dn)
        Ub, dt2 = Ub2, dn
    assert B.check() == 0
    B.fill_guards(Ua, nbr)
    B.fill_guards(Ub, nbr)
    assert torch.equal(Ua, Ub)
