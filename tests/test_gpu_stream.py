"""Host-resident bunches streamed through the device (mhd_stream_*, through the C ABI): the
pipelined update (copy in, update, copy out on three streams over several device slots)
gives the bits of the resident update (mhd_bunch_update on a device copy of the same
state) on owned values, keeps the input's guard values, and is within the per-step bar of
the oracle; with one slot (no overlap) and with a ragged last sub-bunch as well."""
import numpy as np
import pytest

from gpu_util import dev, host, log, make_bunch, rel_err_fields
from paper_2508_09568_amd import workloads as W

pytestmark = pytest.mark.gpu


def _state(name):
    import oracle
    if name == "turb":
        w = W.turbulence(N=64, patch=16)
        L, U, dx, nbr, gam = w.layout, w.U.numpy().copy(), w.dx, w.nbr, w.gamma
    else:
        w = W.uneven(mix=((9, 3), (13, 2), (20, 2)))
        L, U, dx, nbr, gam = w.layout, w.U.numpy().copy(), w.dx, None, w.gamma
    if nbr is not None:
        oracle.fill_guards(U, L.dims, L.g, nbr)
    prm = oracle.Params(gamma=gam)
    dt = oracle.cfl_many(U, L.dims, L.g, dx, prm)
    dt = np.full(L.P, dt.min()) if nbr is not None else dt
    return L, U, np.ascontiguousarray(dx), dt, gam, prm


@pytest.mark.parametrize("name,per,slots,precision,cfg", [("turb", 7, 3, 8, None), ("turb", 16, 1, 8, None),
                                                          ("turb", 5, 2, 4, None), ("ragged", 2, 3, 8, None),
                                                          ("turb", 7, 3, 8, (1, 1, 3)),
                                                          ("ragged", 3, 2, 4, (4, 2, 3))])
def test_streamed_update_matches_resident_update(name, per, slots, precision, cfg):
    """cfg: (tile configuration, predictor mode, solver form) of every sub-bunch and of the
    resident bunch; None keeps the defaults."""
    import oracle
    import torch

    from paper_2508_09568_amd.binding import Stream
    log(f"[gpu] streamed update {name} per={per} slots={slots} precision={precision} cfg={cfg}")
    L, U, dx, dt, gam, prm = _state(name)
    dty = torch.float64 if precision == 8 else torch.float32
    Uh = torch.as_tensor(U).to(dty).pin_memory()
    Uo = torch.full_like(Uh, float("nan")).pin_memory()
    S = Stream(L.dims, per, slots=slots, precision=precision, gamma=gam)
    if cfg is not None:
        S.configure(*cfg)
    assert S.bunches() == (L.P + per - 1) // per
    S.update(Uh, Uo, torch.as_tensor(dt), torch.as_tensor(np.ascontiguousarray(dx).ravel()))
    assert S.check() == 0
    got = Uo.double().numpy()
    # resident update of the same state
    B = make_bunch(L, gam, precision=precision)
    if cfg is not None:
        B.set_tile(cfg[0])
        B.set_predictor(cfg[1])
        B.set_solver_split(cfg[2])
    Ud = Uh.to("cuda")
    Ur = torch.zeros_like(Ud)
    B.update(Ud, Ur, dev(dt), dev(dx))
    assert B.check() == 0
    ref = host(Ur)
    for p in range(L.P):
        assert np.array_equal(L.interior(got, p), L.interior(ref, p)), p
    # guard entries: the input's
    own = np.zeros(L.total, dtype=bool)
    for p in range(L.P):
        L.interior(own, p)[...] = True
    assert np.array_equal(got[~own], Uh.double().numpy()[~own])
    if precision == 8:
        ora = oracle.step_many(U, L.dims, L.g, dt, dx, prm)
        err = rel_err_fields(L, got, ora)
        log(f"    identical to the resident update; vs oracle {err.max():.2e}")
        assert np.all(err <= 1e-12)
