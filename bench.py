#!/usr/bin/env python3
"""Benchmark of the MI355X MHD bunch update (one GPU).

Workload: decaying supersonic MHD turbulence, 512^3 periodic cells as 4096 patches of
32^3 (guard width 3), seeded synthetic initial state.  One timed step = the whole hot
path on every patch: guard exchange, global CFL time step on the device, update
(primitives, EMFs at time n, predictor, HLLD + edge EMFs + conservative/CT update).
The state stays resident in HBM; no host synchronisation inside the timed region.

Prints one JSON line: cell-updates/s for FP64 (headline) with the FP32 result, the
per-kernel HIP-event timings, the roofline of the update and the oracle timed on the
host cores.

Also measured (FP32, "batched vs per-bunch"): an uneven bunch of 3600 patches of four
sizes, each at its own CFL step, as one HIP-graph launch vs per-bunch vs per-patch launches.

  python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--no-fp32] [--no-cpu-baseline]
                  [--no-batched] [--batched-steps 10]
"""
import argparse
import json
import os
import sys
import time

METRIC = "MHD cell-updates/s and % HBM roofline, FP64/FP32, batched vs per-bunch"
PEAK_HBM_GBS = 8000.0
PEAK_VALU_TFLOPS = {8: 78.6, 4: 157.3}     # MI355X vector FP64 / FP32 (published)
UPDATE_KERNELS = ("prim", "edge_emf_n", "predict", "edge", "solve")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# HBM bytes of one FP64 update (every update kernel), measured with rocprofv3 --pmc FETCH_SIZE
# and WRITE_SIZE on the turbulence workload and scaled by the same counters on a plain
# 1 GiB device copy (FETCH_SIZE reads 0.5x there, WRITE_SIZE 1x), for the launch
# configurations the autotuner picks on this workload (within 1 % of each other).  Keyed by
# launch configuration ((tile x, y, z, mode), predictor mode, solver form); valid only for
# the kernel sources and build flags it was measured on: reported as null once they change
# (the hash moves on only with a source change that leaves the machine code of every measured
# kernel as it was).
MEASURED_TRAFFIC = {
    "sources_sha256": "9135b0f9087483f992ccf28c99b7cd38f484677efef61fb8eba63f12cbe72e13",
    "bytes_per_update": {
        "[32, 4, 2, 1]/1/3": 234.06e9,
        "[32, 8, 2, 1]/1/3": 229.05e9,
        "[32, 4, 4, 1]/1/3": 229.34e9,
    },
    "profile": "profiles/mhd_update_turbulence512_pmc.md",
}

def kernel_sources_sha256():
    """Hash of the kernel sources and build flags with comments and blank space removed (a
    comment edit leaves the measured kernels as they were)."""
    import hashlib
    import re
    here = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in ("csrc/mhd_bunch.hip", "csrc/mhd_stages.hpp", "csrc/mhd_physics.hpp", "build.py"):
        with open(os.path.join(here, "paper_2508_09568_amd", f)) as fh:
            text = fh.read()
        if f.endswith(".py"):
            text = re.sub(r"#[^\n]*", "", text)
        else:
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            text = re.sub(r"//[^\n]*", "", text)
        h.update(re.sub(r"\s+", " ", text).encode())
    return h.hexdigest()


def measured_traffic(tile, fused, split):
    m = MEASURED_TRAFFIC
    if m["sources_sha256"] != kernel_sources_sha256():
        return None
    return m["bytes_per_update"].get(f"{list(tile)}/{fused}/{split}")


def algorithmic_bytes_per_cell(n, g, s):
    """Read every padded cell once, write every interior cell once, 8 fields."""
    return 8.0 * s * (((n + 2 * g) / n) ** 3 + 1.0)


def run_precision(w, precision, steps, warmup, flops_per_cell, tile=None, predictor=None,
                  split=None, emf_solver=0):
    import numpy as np
    import torch

    from paper_2508_09568_amd.binding import Bunch

    L = w.layout
    dtype = torch.float64 if precision == 8 else torch.float32
    Ua = w.U.to(dtype=dtype, copy=True)
    Ub = torch.empty_like(Ua)
    B = Bunch(L.dims, g=L.g, precision=precision, gamma=w.gamma, cfl=w.cfl, emf_solver=emf_solver)
    nbr = torch.as_tensor(w.nbr.astype(np.int32)).cuda()
    dx = torch.as_tensor(w.dx).cuda()
    dt = torch.zeros(L.P, dtype=torch.float64, device="cuda")

    def step(a, b):
        B.fill_guards(a, nbr)
        B.cfl(a, dx, dt, global_min=True)
        B.update(a, b, dt, dx)

    # launch configuration: the autotuner times every tile shape (with and without the XCD
    # remap) on this state and keeps the fastest
    B.fill_guards(Ua, nbr)
    B.cfl(Ua, dx, dt, global_min=True)
    cfgs = B.tile_configs()
    if tile is None:
        best, tune_ms = B.autotune(Ua, Ub, dt, dx, reps=2)
        log(f"[bench] autotune: " + ", ".join(f"{c}:{m:.2f}ms" for c, m in zip(cfgs, tune_ms)))
    else:                         # fixed configuration (profiling runs)
        best, tune_ms = tile, [float("nan")] * len(cfgs)
        B.set_tile(tile)
    if predictor is not None:
        B.set_predictor(predictor)
    if split is not None:
        B.set_solver_split(split)
    for _ in range(warmup):
        step(Ua, Ub)
        Ua, Ub = Ub, Ua
    rc = B.check()
    if rc != 0:
        raise RuntimeError(f"device status {rc} after warm-up")

    def timed(fn):
        torch.cuda.synchronize()
        B.profile(True)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        wall0 = time.perf_counter()
        t0.record()
        for _ in range(steps):
            fn()
        t1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        prof = B.profile_read()
        B.profile(False)
        return t0.elapsed_time(t1), wall, prof

    # (1) guard exchange + separate time-step pass + update
    st = [Ua, Ub]

    def sep():
        step(st[0], st[1])
        st.reverse()

    ms_sep, _, _ = timed(sep)
    # (2) guard exchange + update with the next step's time step reduced in its tiles (the
    # same states and time steps bit for bit); the reported step
    cur = [dt, torch.zeros_like(dt)]
    B.fill_guards(st[0], nbr)
    B.cfl(st[0], dx, cur[0], global_min=True)

    def fused():
        B.fill_guards(st[0], nbr)
        B.update_cfl(st[0], st[1], cur[0], dx, nbr, cur[1])
        st.reverse()
        cur.reverse()

    ms, wall, prof = timed(fused)
    Ua, Ub = st
    B.fill_guards(Ua, nbr)       # outside the timed region: guard-filled state for the oracle
    rc = B.check()
    if rc != 0:
        raise RuntimeError(f"device status {rc} after timed steps")
    cells = L.interior_cells
    value = cells * steps / (ms * 1e-3)
    upd_ms = sum(prof[k][0] for k in UPDATE_KERNELS) / steps
    n = int(L.dims[0, 0])
    bpc = algorithmic_bytes_per_cell(n, L.g, precision)
    kern = {k: {"avg_ms": v[0] / max(v[1], 1), "launches": v[1]} for k, v in prof.items()}
    res = {
        "value": value,
        "ms_per_step": ms / steps,
        "separate_time_step": {"value": cells * steps / (ms_sep * 1e-3),
                               "ms_per_step": ms_sep / steps},
        "wall_ms_per_step": 1e3 * wall / steps,
        "update_ms_per_launch": upd_ms,
        "kernels": kern,
        "flops_per_cell": flops_per_cell,
        "bytes_per_cell": bpc,
        "update_tflops": flops_per_cell * cells / (upd_ms * 1e-3) / 1e12,
        "update_hbm_gbs": bpc * cells / (upd_ms * 1e-3) / 1e9,
        "tile": {"chosen": list(cfgs[best]), "fused_predictor": B.predictor(),
                 "predictor_tile": list(B.predictor_modes()[B.predictor()]),
                 "solver_split": B.solver_split(),
                 "tuned_ms": {str(list(c)): (None if m != m else round(m, 3))
                              for c, m in zip(cfgs, tune_ms)}},
        "bunch": B,
    }
    return res


def run_batched(steps, steps_per_patch):
    """Uneven bunch (2000 x 16^3, 1000 x 24^3, 500 x 32^3, 100 x 48^3, FP32, frozen
    guards, each patch at its own CFL step): (A) the whole bunch in one launch set per
    step, all steps in one HIP graph launch; (B) plain launches per same-size bunch of at
    most 300 patches; (C) launches per patch.  Same kernels and per-patch dt, so the three
    give identical bits; reported as cell-updates/s."""
    import numpy as np
    import torch

    from paper_2508_09568_amd import workloads as W
    from paper_2508_09568_amd.binding import Bunch

    t0 = time.perf_counter()
    w = W.uneven(device="cuda", dtype=torch.float32)
    L = w.layout
    log(f"[bench] uneven bunch: {L.P} patches, {L.interior_cells} cells, generated in "
        f"{time.perf_counter() - t0:.1f} s")
    cells = int(L.interior_cells)
    U0 = w.U
    dx = torch.as_tensor(w.dx).cuda()
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    # (A) one bunch, graph of `steps` steps
    B = Bunch(L.dims, g=L.g, precision=4, gamma=w.gamma, cfl=w.cfl)
    Ua, Ub = U0.clone(), U0.clone()        # frozen guards: both buffers carry them
    dt = torch.zeros(L.P, dtype=torch.float64, device="cuda")
    B.cfl(Ua, dx, dt)
    best, tune_ms = B.autotune(Ua, Ub, dt, dx, reps=2)
    B.graph_capture(steps, Ua, Ub, dt, dx, nbr=None, dt_mode=1)
    Ua.copy_(U0)
    B.graph_launch()                       # warm-up replay
    Ua.copy_(U0)
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record()
    B.graph_launch()
    b.record()
    torch.cuda.synchronize()
    ms_a = a.elapsed_time(b)
    if B.check() != 0:
        raise RuntimeError("device status after the batched run")
    res_a = (Ua if steps % 2 == 0 else Ub).clone()
    cfg = B.tile_configs()[best]
    fused = B.predictor()
    split = B.solver_split()
    del B, Ua, Ub
    torch.cuda.empty_cache()
    log(f"[bench] (A) batched graph: {ms_a / steps:.2f} ms/step, tile {cfg}")

    def sub_bunches(groups):
        subs = []
        for idx in groups:
            idx = np.asarray(idx)
            Bs = Bunch(L.dims[idx], g=L.g, precision=4, gamma=w.gamma, cfl=w.cfl)
            Bs.set_tile(best if best < len(Bs.tile_configs()) else 0)
            Bs.set_predictor(fused)
            Bs.set_solver_split(split)
            seg = [U0[int(L.base[p]):int(L.base[p + 1])] for p in idx]
            ua = torch.cat(seg)
            subs.append((idx, Bs, ua, ua.clone(), dx[torch.as_tensor(idx).cuda()].contiguous(),
                         torch.zeros(len(idx), dtype=torch.float64, device="cuda")))
        return subs

    def run_subs(subs, nst):
        cur = [(s[2], s[3]) for s in subs]
        for _ in range(nst):
            nxt = []
            for (idx, Bs, _, _, dxs, dts), (x, y) in zip(subs, cur):
                Bs.cfl(x, dxs, dts)
                Bs.update(x, y, dts, dxs)
                nxt.append((y, x))
            cur = nxt
        return cur

    def compare(subs, cur, ref):
        bad = 0.0
        for (idx, Bs, *_), (x, _) in zip(subs, cur):
            off = 0
            for p in idx[:3]:
                n = int(L.base[p + 1] - L.base[p])
                d = (x[off:off + n] - ref[int(L.base[p]):int(L.base[p + 1])]).abs().max().item()
                bad = max(bad, d)
                off += n
        return bad

    sizes = L.dims[:, 0]
    groups = []
    for n in sorted(set(int(v) for v in sizes)):
        ids = np.nonzero(sizes == n)[0]
        groups += [ids[i:i + 300] for i in range(0, len(ids), 300)]
    subs = sub_bunches(groups)
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record()
    cur = run_subs(subs, steps)
    b.record()
    torch.cuda.synchronize()
    ms_b = a.elapsed_time(b)
    diff_b = compare(subs, cur, res_a)
    log(f"[bench] (B) per-bunch ({len(subs)} bunches): {ms_b / steps:.2f} ms/step, "
        f"max |B - A| on sampled patches {diff_b:.3e}")
    del subs, cur
    torch.cuda.empty_cache()

    subs = sub_bunches([[p] for p in range(L.P)])
    torch.cuda.synchronize()
    run_subs(subs, 1)                      # warm-up (first launches of each handle)
    for s_ in subs:
        s_[2].copy_(U0[int(L.base[s_[0][0]]):int(L.base[s_[0][0] + 1])])
        s_[3].copy_(s_[2])
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record()
    run_subs(subs, steps_per_patch)
    b.record()
    torch.cuda.synchronize()
    ms_c = a.elapsed_time(b)
    log(f"[bench] (C) per-patch ({len(subs)} launches sets/step): "
        f"{ms_c / steps_per_patch:.2f} ms/step")
    del subs
    torch.cuda.empty_cache()
    return {
        "workload": "uneven bunch: 2000 x 16^3 + 1000 x 24^3 + 500 x 32^3 + 100 x 48^3 "
                    "patches (guard 3, frozen guards), turbulence field sampled per patch, "
                    "each patch at its own CFL step; FP32",
        "cell_updates_per_step": cells,
        "steps": steps,
        "batched_graph": {"value": cells * steps / (ms_a * 1e-3), "ms_per_step": ms_a / steps,
                          "launch": "one HIP graph launch for all steps (CFL + update "
                                    "kernels of the whole bunch per step)",
                          "tile": list(cfg), "fused_predictor": fused},
        "per_bunch": {"value": cells * steps / (ms_b * 1e-3), "ms_per_step": ms_b / steps,
                      "bunches": len(groups), "launch": "same-size bunches of <= 300 patches",
                      "max_abs_diff_vs_batched": diff_b},
        "per_patch": {"value": cells * steps_per_patch / (ms_c * 1e-3),
                      "ms_per_step": ms_c / steps_per_patch, "steps": steps_per_patch},
        "speedup_vs_per_bunch": ms_b / ms_a,
        "speedup_vs_per_patch": (ms_c / steps_per_patch) / (ms_a / steps),
    }


def run_lts(w, tile, t_mult, own_only=False):
    """Local time stepping on the benchmark workload (FP64, the tuned launch configuration) to
    t_end = t_mult x the largest power of two not above the smallest patch CFL step, against
    global stepping (guard exchange + global CFL + update) to the same time.  Wall time
    includes the host reading the times.  With own_only, only the eager run with each patch's
    own CFL step (for a kernel trace of its steps)."""
    import numpy as np
    import torch

    from paper_2508_09568_amd import lts
    from paper_2508_09568_amd.binding import Bunch

    L = w.layout
    B = Bunch(L.dims, g=L.g, precision=8, gamma=w.gamma, cfl=w.cfl)
    B.set_tile(B.tile_configs().index(tuple(tile["chosen"])))
    B.set_predictor(tile["fused_predictor"])
    B.set_solver_split(tile["solver_split"])
    U = w.U.to(dtype=torch.float64, copy=True)
    nbr = torch.as_tensor(w.nbr.astype(np.int32)).cuda()
    dx = torch.as_tensor(w.dx).cuda()
    dt = torch.zeros(L.P, dtype=torch.float64, device="cuda")
    B.fill_guards(U, nbr)
    B.cfl(U, dx, dt)
    own = dt.cpu().numpy()
    # time levels use a power-of-two quantum (exact time sums); t_end is a multiple of it
    quantum = 2.0 ** np.floor(np.log2(float(own.min())))
    t_end = t_mult * quantum
    cells = int(np.prod(L.dims[0]))
    if own_only:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Ul, tl, nl, cnt = lts.run(B, U, dx, nbr, t_end, check_every=8)
        torch.cuda.synchronize()
        wall_l = time.perf_counter() - t0
        if B.check() != 0:
            raise RuntimeError("device status after the local-time-stepping run")
        upd_l = int(cnt.sum().item()) * cells
        return {"t_end": t_end, "lts": {"steps": nl, "cell_updates": upd_l, "ms": 1e3 * wall_l,
                                        "cell_updates_per_s": upd_l / wall_l}}
    # global stepping
    Ua, Ub = U.clone(), torch.empty_like(U)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t, nglob = 0.0, 0
    while t < t_end:
        B.fill_guards(Ua, nbr)
        B.cfl(Ua, dx, dt, global_min=True)
        d = min(float(dt[0].item()), t_end - t)
        dt.fill_(d)
        B.update(Ua, Ub, dt, dx)
        Ua, Ub = Ub, Ua
        t = t_end if d >= t_end - t else t + d
        nglob += 1
    torch.cuda.synchronize()
    wall_g = time.perf_counter() - t0
    del Ua, Ub
    upd_g = nglob * L.P * cells
    res = {"t_end": t_end, "patch_dt_max_over_min": float(own.max() / own.min()),
           "global": {"steps": nglob, "cell_updates": upd_g, "ms": 1e3 * wall_g,
                      "cell_updates_per_s": upd_g / wall_g}}
    # local time stepping: each patch at its own CFL step; then with time levels (steps
    # rounded down to a power-of-two quantum x 2^k)
    for key, q in (("lts", 0.0), ("lts_levels", quantum)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Ul, tl, nl, cnt = lts.run(B, U, dx, nbr, t_end, dt_quantum=q, check_every=8)
        torch.cuda.synchronize()
        wall_l = time.perf_counter() - t0
        if B.check() != 0:
            raise RuntimeError("device status after the local-time-stepping run")
        upd_l = int(cnt.sum().item()) * cells
        res[key] = {"dt_quantum": q, "steps": nl,
                    "updates_per_patch": [int(cnt.min().item()), int(cnt.max().item())],
                    "cell_updates": upd_l, "ms": 1e3 * wall_l,
                    "cell_updates_per_s": upd_l / wall_l,
                    "work_ratio": upd_l / upd_g, "time_ratio": wall_l / wall_g}
        # the same run with 16 steps per captured graph (same schedule, same bits)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Ug, tg, ng = lts.run_graph(B, U, dx, nbr, t_end, dt_quantum=q, steps_per_graph=16)
        torch.cuda.synchronize()
        wall_c = time.perf_counter() - t0
        res[key]["graph"] = {"steps_launched": ng, "ms": 1e3 * wall_c,
                             "cell_updates_per_s": upd_l / wall_c,
                             "time_ratio": wall_c / wall_g,
                             "same_bits_as_eager": bool(torch.equal(Ug, Ul) and torch.equal(tg, tl))}
        del Ug, Ul
    return res


def run_stream(w, tile, per_bunch=256):
    """The 512^3 turbulence (FP32) held in page-locked host memory and streamed through the
    device for one update: sub-bunches of `per_bunch` patches, copy in / update / copy out on
    three streams over 3 device slots (overlapped) and over 1 slot (serial).  Time on the
    current stream from the first copy in to the last copy out (the PCIe-inclusive rate)."""
    import numpy as np
    import torch

    from paper_2508_09568_amd.binding import Bunch, Stream

    L = w.layout
    nbr = torch.as_tensor(w.nbr.astype(np.int32)).cuda()
    dx = torch.as_tensor(w.dx).cuda()
    B = Bunch(L.dims, g=L.g, precision=4, gamma=w.gamma, cfl=w.cfl)
    Ud = w.U.to(dtype=torch.float32, copy=True)
    dt = torch.zeros(L.P, dtype=torch.float64, device="cuda")
    B.fill_guards(Ud, nbr)
    B.cfl(Ud, dx, dt, global_min=True)
    cfg = B.tile_configs().index(tuple(tile["chosen"]))
    B.set_tile(cfg)
    B.set_predictor(tile["fused_predictor"])
    B.set_solver_split(tile["solver_split"])
    Ur = torch.empty_like(Ud)
    B.update(Ud, Ur, dt, dx)
    Uh = torch.empty(Ud.numel(), dtype=torch.float32, pin_memory=True)
    Uh.copy_(Ud)
    Uo = torch.empty_like(Uh).pin_memory()
    dth, dxh = dt.cpu(), dx.reshape(-1).cpu()
    del Ud
    torch.cuda.empty_cache()
    nbytes = 2 * Uh.numel() * 4
    cells = int(L.interior_cells)
    out = {"workload": f"512^3 turbulence, FP32, in page-locked host memory; sub-bunches of "
                       f"{per_bunch} patches", "bytes_per_update": nbytes}
    for slots in (3, 1):
        S = Stream(L.dims, per_bunch, slots=slots, precision=4, gamma=w.gamma, cfl=w.cfl)
        S.configure(cfg, tile["fused_predictor"], tile["solver_split"])
        S.update(Uh, Uo, dth, dxh)            # warm-up
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        S.update(Uh, Uo, dth, dxh)
        b.record()
        torch.cuda.synchronize()
        if S.check() != 0:
            raise RuntimeError("device status after the streamed update")
        ms = a.elapsed_time(b)
        out[f"slots_{slots}"] = {"ms": ms, "cell_updates_per_s": cells / (ms * 1e-3),
                                 "pcie_gbs": nbytes / (ms * 1e-3) / 1e9,
                                 "sub_bunches": S.bunches()}
        del S
        torch.cuda.empty_cache()
    # sampled patches against the resident update
    ref = Ur.cpu()
    bad = 0.0
    for p in (0, L.P // 2, L.P - 1):
        a0, a1 = int(L.base[p]), int(L.base[p + 1])
        own = _owned_in_block(L, p)
        bad = max(bad, float(np.abs(Uo.numpy()[a0:a1][own] - ref.numpy()[a0:a1][own]).max()))
    out["max_abs_diff_vs_resident"] = bad
    # no pipeline: the whole state copied in, updated, copied out, one after the other
    Ud = torch.empty(Uh.numel(), dtype=torch.float32, device="cuda")
    Uo2 = torch.empty_like(Ud)
    dtd = dth.cuda()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    Ud.copy_(Uh, non_blocking=True)
    B.update(Ud, Uo2, dtd, dx)
    Uo.copy_(Uo2, non_blocking=True)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    out["whole_state_serial"] = {"ms": ms, "cell_updates_per_s": cells / (ms * 1e-3),
                                 "launch": "copy the whole state in, update, copy it out"}
    del Ud, Uo2
    torch.cuda.empty_cache()
    out["pipeline_speedup_vs_serial"] = out["whole_state_serial"]["ms"] / out["slots_3"]["ms"]
    out["overlap_speedup"] = out["slots_1"]["ms"] / out["slots_3"]["ms"]
    return out


def _owned_in_block(L, p):
    """Boolean mask of patch p's owned entries inside its own block of the state."""
    import numpy as np
    from paper_2508_09568_amd import workloads as W
    Lp = W.Layout(L.dims[p][None], L.g)
    m = np.zeros(Lp.total, dtype=bool)
    Lp.interior(m, 0)[...] = True
    return m


def cpu_baseline(block):
    """The oracle's step on a corner block of block^3 patches of the same seeded turbulence
    (same cell size and patch shape), generated on the host; guards filled by the oracle
    (periodic faces of the full domain become zero-gradient boundaries of the block) and one
    common dt from the oracle's CFL, as in the GPU step.  Only the update is timed."""
    import numpy as np

    import oracle
    from paper_2508_09568_amd import workloads as W

    w = W.turbulence(grid=(block, block, block))
    L = w.layout
    U = w.U.numpy()
    prm = oracle.Params(gamma=w.gamma, cfl=w.cfl)
    oracle.fill_guards(U, L.dims, L.g, w.nbr)
    dt = float(np.min(oracle.cfl_many(U, L.dims, L.g, w.dx, prm)))
    t0 = time.perf_counter()
    oracle.step_many(U, L.dims, L.g, np.full(L.P, dt), w.dx, prm)
    el = time.perf_counter() - t0
    cells = int(np.prod(L.dims.astype(np.int64), axis=1).sum())
    nth = oracle.threads()
    # one thread: the first 64 patches of the same block
    n1 = min(64, L.P)
    end = int(L.base[n1])
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.step_many(np.ascontiguousarray(U[:end]), L.dims[:n1], L.g, np.full(n1, dt),
                         w.dx[:n1], prm)
        el1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(nth)
    cells1 = int(np.prod(L.dims[:n1].astype(np.int64), axis=1).sum())
    return {"value": cells / el, "unit": "cell-updates/s", "cores": nth, "kind": "oracle",
            "sample": f"{L.P} patches of 32^3 ({block}^3 corner block of the 512^3 turbulence, "
                      f"FP64), one update: {cells} cell-updates in {el:.2f} s on {nth} threads "
                      f"(~{el * nth:.0f} thread-seconds)",
            "single_thread": {"value": cells1 / el1, "unit": "cell-updates/s", "cores": 1,
                              "sample": f"the first {n1} patches of that block, one update: "
                                        f"{cells1} cell-updates in {el1:.2f} s on 1 thread"},
            "cpu": _cpu_model()}


def cpu_baseline_uneven():
    """The oracle's step of the whole uneven bunch (3600 patches of four sizes, each at its own
    CFL step, frozen guards), in FP64 on all host threads.  The state is generated on the GPU
    by the same generator as the GPU run and copied to the host."""
    import numpy as np
    import torch

    import oracle
    from paper_2508_09568_amd import workloads as W

    w = W.uneven(device="cuda", dtype=torch.float64)
    L, dx, prm = w.layout, w.dx, oracle.Params(gamma=w.gamma, cfl=w.cfl)
    U = w.U.cpu().numpy()
    del w
    torch.cuda.empty_cache()
    dt = oracle.cfl_many(U, L.dims, L.g, dx, prm)
    t0 = time.perf_counter()
    oracle.step_many(U, L.dims, L.g, dt, dx, prm)
    el = time.perf_counter() - t0
    cells = int(L.interior_cells)
    nth = oracle.threads()
    return {"value": cells / el, "unit": "cell-updates/s", "cores": nth, "kind": "oracle",
            "sample": f"one step of all {L.P} patches ({cells} cell-updates, FP64, own CFL "
                      f"steps) in {el:.2f} s on {nth} threads"}


def run_adjoint(reps):
    """Adjoint workload (64^3 periodic as 8 patches of 32^3, FP64, fast wave + noise): 20 steps
    at the fixed time step of the noise-free state, checkpoint every 5; gradient of the L2
    misfit of the final density against the seeded target.  Times the forward rollout alone
    and forward + backward (HIP events on the current stream, mean of `reps`)."""
    import numpy as np
    import torch

    from paper_2508_09568_amd import workloads as W
    from paper_2508_09568_amd.autodiff import rollout
    from paper_2508_09568_amd.binding import Bunch

    nsteps, every = 20, 5
    w = W.adjoint_case()
    L = w.layout
    B = Bunch(L.dims, g=L.g, precision=8, gamma=w.gamma, cfl=w.cfl)
    B.adjoint_bind(w.nbr)
    nbr = torch.as_tensor(w.nbr.astype(np.int32)).cuda()
    dx = torch.as_tensor(w.dx).cuda()
    Uc = torch.as_tensor(W.adjoint_case(noise=0.0).U).cuda()
    dt = torch.zeros(L.P, dtype=torch.float64, device="cuda")
    B.fill_guards(Uc, nbr)
    B.cfl(Uc, dx, dt, global_min=True)
    dts = dt.expand(nsteps, L.P).contiguous()
    mask = np.zeros(L.total)
    for p in range(L.P):
        L.interior(mask, p)[0] = 1.0
    mask = torch.as_tensor(mask).cuda()
    with torch.no_grad():
        rho_t = rollout(torch.as_tensor(W.adjoint_case(noise_seed=6).U).cuda(), B, nbr, dts, dx,
                        every) * mask
    U0 = torch.as_tensor(w.U).cuda()

    def fwd():
        with torch.no_grad():
            return rollout(U0, B, nbr, dts, dx, every)

    def fwd_bwd():
        x = U0.clone().requires_grad_(True)
        r = rollout(x, B, nbr, dts, dx, every) * mask
        (0.5 * ((r - rho_t) ** 2).sum()).backward()
        return x.grad

    out = {}
    for key, fn in (("forward", fwd), ("forward_backward", fwd_bwd)):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        out[key + "_ms"] = a.elapsed_time(b) / reps
    if B.check() != 0:
        raise RuntimeError("device status after the adjoint runs")
    cells = int(L.interior_cells)
    return {"workload": "64^3 periodic as 8 patches of 32^3, FP64, fast wave + noise; 20 steps "
                        "at fixed dt, checkpoint every 5; gradient of the L2 density misfit",
            "steps": nsteps, "checkpoint_every": every, **out,
            "backward_over_forward": out["forward_backward_ms"] / out["forward_ms"] - 1.0,
            "forward_cell_updates_per_s": cells * nsteps / (out["forward_ms"] * 1e-3)}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-block", type=int, default=8,
                    help="CPU baseline sample: a corner block of this many patches per side")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--tile", type=int, default=None,
                    help="use this launch configuration instead of autotuning")
    ap.add_argument("--predictor", type=int, default=None,
                    help="force the predictor mode: 0 staged kernels, k >= 1 fused tile kernel "
                         "with the k-th tile shape (for 3D: 1 = 8x8x4, 2 = 34x4x2)")
    ap.add_argument("--split", type=int, default=None, choices=(0, 1, 2, 3),
                    help="force the solver form: one-phase (0), two-phase (1), edge pass (2), edge-line pass (3)")
    ap.add_argument("--fp32-only", action="store_true",
                    help="skip the FP64 run (profiling of the FP32 kernels)")
    ap.add_argument("--batched-steps", type=int, default=10)
    ap.add_argument("--no-stream", action="store_true",
                    help="skip the host-resident streamed update")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint workload's forward / backward timing")
    ap.add_argument("--no-uct-hlld", action="store_true",
                    help="skip the FP64 step with the UCT-HLLD edge EMF (emf_solver 1)")
    ap.add_argument("--uct-hlld-only", action="store_true",
                    help="only the FP64 step with the UCT-HLLD edge EMF (for a kernel trace; "
                         "--tile / --predictor / --split as for the main step), then exit")
    ap.add_argument("--no-lts", action="store_true",
                    help="skip the local-time-stepping run")
    ap.add_argument("--lts-span", type=float, default=8.0,
                    help="local-time-stepping run to this many smallest patch CFL steps")
    ap.add_argument("--lts-only", action="store_true",
                    help="only the FP64 local-time-stepping run with each patch's own CFL step "
                         "(eager launches, for a kernel trace), in the launch configuration "
                         "--tile / --predictor / --split, then exit")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the adjoint workload's forward and forward + backward timing "
                         "(for a kernel trace), then exit")
    ap.add_argument("--bw-probe", action="store_true",
                    help="only measure the device's memory ceilings (fill, sum and copy of "
                         "4 GiB FP64, HIP events, 10 repetitions each) and exit")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run 5 plain device-to-device copies of this many bytes (HBM "
                         "counter calibration under rocprofv3 --pmc) and exit")
    args = ap.parse_args()
    if args.adjoint_only:
        print(json.dumps({"adjoint_only": run_adjoint(3)}), flush=True)
        return
    if args.bw_probe:
        import torch
        nbytes = 4 << 30
        x = torch.full((nbytes // 8,), 1.0, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)

        def per_call(f, reps=10):
            f()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                f()
            b.record()
            torch.cuda.synchronize()
            return a.elapsed_time(b) / reps / 1e3

        tw, tr, tc = per_call(lambda: x.fill_(3.0)), per_call(lambda: x.sum()), \
            per_call(lambda: y.copy_(x))
        print(json.dumps({"bw_probe_bytes": nbytes, "write_tb_s": nbytes / tw / 1e12,
                          "read_tb_s": nbytes / tr / 1e12,
                          "copy_read_plus_write_tb_s": 2 * nbytes / tc / 1e12}), flush=True)
        return
    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the update has no multi-GPU path in this "
              "build (patches would shard by contiguous blocks with a guard exchange per "
              "step; not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import oracle
    from paper_2508_09568_amd import workloads as W

    torch.cuda.init()
    dev = torch.cuda.get_device_name(0)
    log(f"[bench] device {dev}; generating turbulence 512^3 as 4096 x 32^3 (seed 3)")
    t0 = time.perf_counter()
    w = W.turbulence(device="cuda")
    log(f"[bench] generated in {time.perf_counter() - t0:.1f} s")
    # algorithmic arithmetic per cell-update (oracle op count on one patch of the workload)
    p0 = w.U[int(w.layout.base[0]):int(w.layout.base[1])].cpu().numpy()
    ops = oracle.ops_per_cell(p0, w.layout.dims[0], w.layout.g, 1e-4, w.dx[0],
                              oracle.Params(gamma=w.gamma))
    flops = float(ops[:4].sum())
    ops1 = oracle.ops_per_cell(p0, w.layout.dims[0], w.layout.g, 1e-4, w.dx[0],
                               oracle.Params(gamma=w.gamma, emf_solver=1))
    flops_uct_hlld = float(ops1[:4].sum())

    def uct_hlld_summary(r):
        return {"emf_solver": 1, "value": r["value"], "ms_per_step": r["ms_per_step"],
                "update_ms_per_launch": r["update_ms_per_launch"],
                "flops_per_cell": flops_uct_hlld,
                "alu_frac": r["update_tflops"] / PEAK_VALU_TFLOPS[8],
                "kernels_ms": {k: v["avg_ms"] for k, v in r["kernels"].items()},
                "tile": r["tile"]}

    if args.uct_hlld_only:
        rh = run_precision(w, 8, args.steps, args.warmup, flops_uct_hlld, args.tile,
                           args.predictor, args.split, emf_solver=1)
        print(json.dumps({"uct_hlld_only": uct_hlld_summary(rh)}), flush=True)
        return

    if args.lts_only:
        from paper_2508_09568_amd.binding import Bunch
        if args.tile is None or args.predictor is None or args.split is None:
            sys.exit("--lts-only needs --tile, --predictor and --split")
        L = w.layout
        cfgs = Bunch(L.dims, g=L.g, precision=8, gamma=w.gamma, cfl=w.cfl).tile_configs()
        tile = {"chosen": list(cfgs[args.tile]), "fused_predictor": args.predictor,
                "solver_split": args.split}
        res = run_lts(w, tile, args.lts_span, own_only=True)
        print(json.dumps({"lts_only": res, "tile": tile}), flush=True)
        return
    if args.fp32_only:
        r32 = run_precision(w, 4, args.steps, args.warmup, flops, args.tile, args.predictor,
                            args.split)
        print(json.dumps({"fp32_only": {"value": r32["value"], "ms_per_step": r32["ms_per_step"],
                                        "kernels_ms": {k: v["avg_ms"]
                                                       for k, v in r32["kernels"].items()},
                                        "tile": r32["tile"]}}), flush=True)
        return
    log(f"[bench] FP64: warmup {args.warmup}, timed {args.steps} steps")
    r64 = run_precision(w, 8, args.steps, args.warmup, flops, args.tile, args.predictor,
                        args.split)
    log(f"[bench] FP64 {r64['value']:.4e} cell-updates/s, {r64['ms_per_step']:.2f} ms/step "
        f"(separate time-step pass: {r64['separate_time_step']['ms_per_step']:.2f} ms/step)")
    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] CPU baseline: oracle on {args.cpu_block}^3 patches")
        cpu = cpu_baseline(args.cpu_block)
        log(f"[bench] oracle {cpu['value']:.4e} cell-updates/s on {cpu['cores']} threads")
        log(f"[bench] oracle {cpu['single_thread']['value']:.4e} cell-updates/s on 1 thread")
    r64.pop("bunch")
    torch.cuda.empty_cache()
    r32 = None
    if not args.no_fp32:
        log(f"[bench] FP32: warmup {args.warmup}, timed {args.steps} steps")
        r32 = run_precision(w, 4, args.steps, args.warmup, flops, args.tile, args.predictor,
                            args.split)
        r32.pop("bunch")
        log(f"[bench] FP32 {r32['value']:.4e} cell-updates/s, {r32['ms_per_step']:.2f} ms/step")

    uct_hlld = None
    if not args.no_uct_hlld:
        torch.cuda.empty_cache()
        log(f"[bench] FP64 with the UCT-HLLD edge EMF: warmup {args.warmup}, timed {args.steps} "
            f"steps")
        rh = run_precision(w, 8, args.steps, args.warmup, flops_uct_hlld, args.tile,
                           args.predictor, args.split, emf_solver=1)
        rh.pop("bunch")
        uct_hlld = uct_hlld_summary(rh)
        uct_hlld["time_vs_uct_hll"] = rh["ms_per_step"] / r64["ms_per_step"]
        log(f"[bench] UCT-HLLD {rh['value']:.4e} cell-updates/s, {rh['ms_per_step']:.2f} ms/step "
            f"({uct_hlld['time_vs_uct_hll']:.2f}x the UCT-HLL step)")

    batched = None
    if not args.no_batched:
        torch.cuda.empty_cache()
        batched = run_batched(args.batched_steps, 2)
        log(f"[bench] batched vs per-bunch {batched['speedup_vs_per_bunch']:.2f}x, "
            f"vs per-patch {batched['speedup_vs_per_patch']:.2f}x")

    stream = None
    if not args.no_stream and r32 is not None:
        torch.cuda.empty_cache()
        stream = run_stream(w, r32["tile"])
        log(f"[bench] streamed from host: {stream['slots_3']['ms']:.1f} ms with 3 slots, "
            f"{stream['slots_1']['ms']:.1f} ms with 1 ({stream['slots_3']['pcie_gbs']:.1f} GB/s "
            f"over PCIe), max diff vs resident {stream['max_abs_diff_vs_resident']:.1e}")
    adj = None
    if not args.no_adjoint:
        torch.cuda.empty_cache()
        adj = run_adjoint(3)
        log(f"[bench] adjoint workload: forward {adj['forward_ms']:.1f} ms, forward + backward "
            f"{adj['forward_backward_ms']:.1f} ms")
    if cpu is not None and not args.no_batched:
        torch.cuda.empty_cache()
        log("[bench] CPU baseline: oracle step of the uneven bunch")
        cpu["uneven_bunch_step"] = cpu_baseline_uneven()
        log(f"[bench] oracle {cpu['uneven_bunch_step']['value']:.4e} cell-updates/s on the uneven "
            f"bunch")

    lts_res = None
    if not args.no_lts:
        torch.cuda.empty_cache()
        lts_res = run_lts(w, r64["tile"], args.lts_span)
        for key in ("lts", "lts_levels"):
            r = lts_res[key]
            log(f"[bench] {key} to {lts_res['t_end']:.3e}: {r['steps']} steps, {r['ms']:.1f} "
                f"ms, work {r['work_ratio']:.2f}x and time {r['time_ratio']:.2f}x of global "
                f"stepping ({lts_res['global']['steps']} steps, "
                f"{lts_res['global']['ms']:.1f} ms)")
            log(f"[bench] {key} in graphs of 16 steps: {r['graph']['ms']:.1f} ms, time "
                f"{r['graph']['time_ratio']:.2f}x of global stepping, same bits "
                f"{r['graph']['same_bits_as_eager']}")

    peak = PEAK_VALU_TFLOPS[8]
    out = {
        "metric": METRIC,
        "value": r64["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "decaying supersonic MHD turbulence, 512^3 periodic cells as 4096 "
                        "patches of 32^3, guard 3, seeded velocity field (rms Mach 4); "
                        "step = guard exchange + update with the next global CFL step reduced "
                        "in the update's tiles",
            "patches": int(w.layout.P), "patch_cells": [32, 32, 32], "guard": 3,
            "cell_updates_per_step": int(w.layout.interior_cells),
            "device": dev,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "mhd_bunch_update (launches: " + ", ".join(UPDATE_KERNELS) + ")",
            "achieved": r64["update_tflops"],
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": r64["update_tflops"] / peak,
            "traffic": measured_traffic(r64["tile"]["chosen"], r64["tile"]["fused_predictor"],
                                        r64["tile"]["solver_split"]),
            "traffic_note": "HBM bytes per update from rocprofv3 FETCH_SIZE/WRITE_SIZE, scaled "
                            "by a plain copy; null when the kernels or the launch configuration "
                            "differ from the profiled ones",
            "flops_per_cell": flops,
        },
        "hbm": {
            "achieved": r64["update_hbm_gbs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": r64["update_hbm_gbs"] / PEAK_HBM_GBS,
            "bytes_per_cell": r64["bytes_per_cell"],
        },
        "kernels_ms": {k: v["avg_ms"] for k, v in r64["kernels"].items()},
        "separate_time_step": r64["separate_time_step"],
        "tile": r64["tile"],
        "fp32": None if r32 is None else {
            "value": r32["value"], "ms_per_step": r32["ms_per_step"],
            "separate_time_step": r32["separate_time_step"],
            "update_ms_per_launch": r32["update_ms_per_launch"],
            "alu_frac": r32["update_tflops"] / PEAK_VALU_TFLOPS[4],
            "hbm_frac": r32["update_hbm_gbs"] / PEAK_HBM_GBS,
            "kernels_ms": {k: v["avg_ms"] for k, v in r32["kernels"].items()},
            "tile": r32["tile"],
        },
        "uct_hlld": uct_hlld,
        "batched": batched,
        "local_time_stepping": lts_res,
        "adjoint": adj,
        "host_streaming": stream,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
