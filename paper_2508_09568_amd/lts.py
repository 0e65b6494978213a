"""Local time stepping over a bunch: every patch advances with its own time step and fills
its guards at its own time from the neighbours' two time slices (the asynchronous patch
updates of the paper's §2.2 "DISPATCH"; guard interpolation between patch times, §3.1).
Each step is one `mhd_bunch_lts_step` call; the host only reads the patch times to stop."""
from __future__ import annotations

import torch


def run_graph(bunch, U, dx, nbr, t_end, dt_fixed=None, dt_quantum=0.0, steps_per_graph=16,
              max_steps=1_000_000):
    """The same run with `steps_per_graph` local time steps captured in one HIP graph
    (mhd_bunch_lts_graph_capture), launched until every patch has reached t_end; the host reads
    the device status and the times after each launch.  Same results as run(), bit for bit.
    Returns (U at t_end, t, steps launched)."""
    from .binding import MhdError
    P = bunch.P
    dev = U.device
    Ua, Up = U.clone(), U.clone()
    t = torch.zeros(P, dtype=torch.float64, device=dev)
    tp = torch.zeros(P, dtype=torch.float64, device=dev)
    dt = torch.zeros(P, dtype=torch.float64, device=dev)
    bunch.lts_graph_capture(steps_per_graph, Ua, None, Up, t, tp, dt, dx, nbr, t_end,
                            dt_fixed=dt_fixed, dt_quantum=dt_quantum)
    n = 0
    while n < max_steps:
        bunch.graph_launch()
        n += steps_per_graph
        rc = bunch.check()
        if rc != 0:
            raise MhdError(rc, "lts.run_graph: device status after step %d" % n)
        if bool((t >= t_end).all()):
            return Ua, t, n
    raise RuntimeError("lts.run_graph: step limit reached")


def run(bunch, U, dx, nbr, t_end, dt_fixed=None, dt_quantum=0.0, check_every=16,
        max_steps=1_000_000):
    """Advance the state tensor U (guards filled or not) to t_end; dt_quantum > 0 rounds every
    step down to dt_quantum x 2^k (time levels).  Every `check_every` steps the host reads
    the device status (raising on a non-physical state, a bad neighbour table or a step that
    is not finite and > 0) and the patch times.  Returns (U at t_end, t (all t_end), number
    of steps in which some patch advanced, updates per patch); the launches after the last
    such step (at most check_every - 1, none of which changes anything) are not counted."""
    from .binding import MhdError
    P = bunch.P
    dev = U.device
    Ua, Up = U.clone(), U.clone()
    t = torch.zeros(P, dtype=torch.float64, device=dev)
    tp = torch.zeros(P, dtype=torch.float64, device=dev)
    dt = torch.zeros(P, dtype=torch.float64, device=dev)
    count = torch.zeros(P, dtype=torch.int64, device=dev)
    nwork = torch.zeros((), dtype=torch.int64, device=dev)
    n = 0
    while n < max_steps:
        bunch.lts_step(Ua, None, Up, t, tp, dt, dx, nbr, t_end, dt_fixed=dt_fixed,
                       dt_quantum=dt_quantum)
        adv = dt > 0
        count += adv
        nwork += adv.any()
        n += 1
        if n % check_every == 0:
            rc = bunch.check()
            if rc != 0:
                raise MhdError(rc, "lts.run: device status after step %d" % n)
            if bool((t >= t_end).all()):
                break
    else:
        raise RuntimeError("lts.run: step limit reached")
    return Ua, t, int(nwork.item()), count
