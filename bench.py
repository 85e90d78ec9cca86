#!/usr/bin/env python3
"""Throughput of the PIC hot path on one MI355X.

Workload (default): periodic 1024 x 256 grid, dx = 0.1 c/omega_pe, pair plasma
at gamma0 = 40 with T = 0.01 m c^2, 64 particles/cell/species (33,554,432
particles), cubic (order-3) shape, CFL 1.0, theta = 0.6, field CG to 1e-8.
One step = gather + Boris push + move + Esirkepov deposit of every particle,
tile re-binning, the current reduction and the implicit field solve (RHS of
Eq. (7), CG, update of Eqs. (5)-(6)).

The timed form is the FP32 particle path (FP64 fields and CG) with the learned
CG aid: the network is trained on the (b, dB) pairs of the first steps (solved
by plain CG), then every timed step starts the field solve from x0 = N(b) and
runs flexible PCG to the same 1e-8 relative residual. Training is a one-time
set-up, timed and reported on its own. The same workload with plain CG in the
FP32 form and the plain FP64 form (on a schedule tuned for it) are timed on
the same GPU beside it. The schedule (tile shape, work-groups per tile,
field-solve work-groups, reordering period) is autotuned first; the timed
steps are replayed from captured two-step HIP graphs (--no-graph: plain
launches). The timed steps follow 300 untimed ones (--warmup): by then the
numerical Cherenkov instability of the drifting plasma has saturated, and the
timed steps see the hot, bunched state in which a 2000-step run spends most
of its steps (the particle kernel is ~40% slower there than at the cold
start); the tuner's candidates get the same warm-up, and the learned aid is
trained on the pairs of the first steps, before it. Inputs are synthetic
(seeded Maxwell-Juettner load) and resident in HBM before the timed region.
Further legs: the 48-run sweep in one context, the large single-GPU share
(8192 x 2048, 2.1e9 particles), the shock workload (walls, injection), the
network's application rate and the CPU oracle on a strip of the workload.

Prints one JSON line.
"""
import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic HBM bytes per particle-step: read + write of the particle state
BYTES_PER_PARTICLE = {"fp32": 2 * (4 + 5 * 4), "fp64": 2 * (4 + 5 * 8)}
HBM_PEAK_GBS = 8000.0

CONFIGS = {
    # name: nx, ny, ppc, gamma0, order, cfl, theta
    "c2": dict(nx=1024, ny=256, ppc=64, gamma0=40.0, order=3, cfl=1.0, theta=0.6,
               label="periodic 1024x256, pair gamma0=40, 64 ppc/species, order 3, "
                     "CFL 1.0, theta 0.6"),
    "c1": dict(nx=64, ny=64, ppc=16, gamma0=20.0, order=1, cfl=1.0, theta=0.6,
               label="periodic 64x64, pair gamma0=20, 16 ppc/species, order 1, "
                     "CFL 1.0, theta 0.6"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_leg(name, fn):
    """Run one secondary leg of the benchmark: its result, or {"error": ...}
    when it raises (the line still prints the timed form's figures). The
    failed leg's context, and with it its workspace, is released before the
    next leg allocates."""
    try:
        return fn()
    except Exception as e:
        log(f"bench: {name} failed: {type(e).__name__}: {e}")
        err = {"error": f"{type(e).__name__}: {e}"}
    gc.collect()
    return err


def measured_traffic(precision, tile, tile_split, order, n_particles, sort_every=0, warmup=0):
    """HBM bytes per launch of the particle kernel from the committed counter
    record (rocprofv3 FETCH_SIZE and WRITE_SIZE, each scaled by what the same
    counter reads for a copy of known size), or None when the kernel sources or
    the launch configuration differ from the ones the counters were taken on."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.traffic.json")):
        with open(path) as f:
            rec = json.load(f)
        cfg = rec["config"]
        # the warm-up length counts: the hot, bunched plasma after the
        # instability saturates moves other bytes than the cold start
        if (cfg["precision"], list(cfg["tile"]), cfg["tile_split"], cfg["order"],
                cfg["particles"], cfg.get("sort_every", 0),
                cfg.get("warmup", 0)) != (precision, list(tile), tile_split, order, n_particles,
                                          sort_every, warmup):
            continue
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != rec["sources_sha256"]:
            continue
        return rec["traffic_bytes"], os.path.relpath(path, ROOT)
    return None, None


GRAPH = True    # pic_step replays captured two-step HIP graphs (--no-graph: plain launches)
SORT = 0        # pic_options.sort_every of the timed forms (autotuned, or --sort-every)
# (tile shape, reordering period) candidates of the 48-run sweep
SWEEP_SCHEDULES = (((16, 16), 0), ((4, 32), 8), ((8, 16), 8))
EXF = 0.5       # inbox slots per tile (fraction of the tile's slots): narrow tiles in the
                # flow direction exchange up to a quarter of their particles per step
SLACK = 0.5     # tile slots over ppc*cells: once the numerical Cherenkov instability has
                # saturated (near step 300) the densities bunch and a tile of the default
                # 0.25 overflows within the 2000-step run


def make_sim(pic, cfg, load, precision, tile, cg_blocks=0, tile_split=0, solver="cg",
             form="collapsed", slots=0, sort_every=None):
    from synth import loads
    Q = loads.macro_charge(cfg["gamma0"], 0.1, 0.1, cfg["ppc"])
    run = pic.run_desc(cfg["nx"], cfg["ny"], 0.1, cfg["cfl"], cfg["theta"], cfg["order"],
                       [(-Q, Q, cfg["ppc"]), (Q, Q, cfg["ppc"])], cg_rtol=1e-8, cg_maxit=200)
    sim = pic.Sim([run], pic.make_options(precision, tile=tile, diag_every=0,
                                          cg_blocks=cg_blocks, track_ids=False,
                                          tile_split=tile_split, solver=solver,
                                          learned_form=form, precond_slots=slots,
                                          graph=GRAPH,
                                          sort_every=SORT if sort_every is None else sort_every,
                                          exchange_frac=EXF, slack=SLACK))
    for s in range(2):
        d = load[s]
        sim.load_particles(0, s, d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"], d["uz"])
    return sim


def time_form(pic, torch, cfg, load, precision, tile, steps, warmup, cg_blocks=0, tile_split=0,
              learned=None, retune=False, sort_every=None):
    """learned: None (plain CG) or dict(form, pairs, epochs, lr): collect that
    many pairs with plain CG in the first steps, train, then take the learned
    path for the warm-up and the timed steps (as a run would: trained on
    the first steps' pairs the network needs 3 iterations per component after
    the instability has saturated, trained on pairs taken there 4)."""
    solver = "learned" if learned else "cg"
    sim = make_sim(pic, cfg, load, precision, tile, cg_blocks, tile_split, solver,
                   learned["form"] if learned else "collapsed",
                   learned["pairs"] if learned else 0, sort_every)
    n_part = 2 * cfg["nx"] * cfg["ny"] * cfg["ppc"]
    train = None
    if learned:
        sim.precond_use(False)
        sim.precond_collect(True)
        sim.step(learned["pairs"])
        sim.precond_collect(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr = sim.precond_train(learned["epochs"], learned["lr"])
        train = dict(tr, seconds=time.perf_counter() - t0, pairs=learned["pairs"],
                     epochs=learned["epochs"], form=learned["form"])
        sim.precond_use(True)
        if retune:
            # the learned solver has its own best field-solve grid: re-tune it
            # on this context (the work-groups per tile stay as chosen)
            train["retune"] = sim.tune(2, splits=(max(1, tile_split),))
    if warmup:
        sim.step(warmup)
    torch.cuda.synchronize()
    # event timing switches graph replay off, so with graphs the timed region
    # runs without events and a few plain steps afterwards give the breakdown
    sim.timing(not GRAPH)
    t0 = time.perf_counter()
    rc = sim.step_async(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if rc not in (0,):
        raise RuntimeError(f"pic_step returned {pic.STATUS.get(rc, rc)}")
    replays = sim.get_timing()["graph_replays"]
    if GRAPH:
        sim.timing(True)
        sim.step(min(steps, 10))
        steps_t = min(steps, 10)
    else:
        steps_t = steps
    tim = sim.get_timing()
    st = sim.step(0)
    sim.timing(False)
    sim.close()
    ms = (t1 - t0) * 1e3 / steps
    push = tim["push"]
    push_ms = push["ms"] / max(1, push["launches"])
    return dict(ms_per_step=ms, particle_steps_per_s=n_part / (ms * 1e-3),
                push_ms=push_ms, field_solve_ms=tim["field_solve"]["ms"] / max(1, steps_t),
                rebin_ms=tim["rebin"]["ms"] / max(1, steps_t),
                current_sum_ms=tim["current_sum"]["ms"] / max(1, steps_t),
                sort_ms_per_step=tim["sort"]["ms"] / max(1, steps_t),
                graph_replays=replays,
                cg_iters=st[0]["iters"], learned_iters=st[0]["learned_iters"],
                fallback=st[0]["fallback"], relres=st[0]["relres"], n_particles=n_part,
                train=train)


def batched_sweep(pic, torch, steps, warmup, seq_steps=3, learned_pairs=8, learned_epochs=50):
    """The 48-run sweep table in one context (FP32 particles) against the same
    runs launched one context at a time; aggregate particle-steps/s."""
    from synth import configs, loads
    table = configs.sweep_runs()
    descs = []
    for t in table:
        Q = loads.macro_charge(t["gamma0"], t["dx"], t["dx"], t["ppc"])
        descs.append(pic.run_desc(t["nx"], t["ny"], t["dx"], t["cfl"], t["theta"], t["order"],
                                  [(-Q, Q, t["ppc"]), (Q, Q, t["ppc"])], cg_rtol=1e-8))

    def load_run(sim, r, t):
        # the device loader generates the same seeded items as the host generator
        for s in range(2):
            sim.load_plasma(r, s, t["ppc"], t["gamma0"], t["T"], t["seed"])
    n_part = sum(2 * t["nx"] * t["ny"] * t["ppc"] for t in table)

    def timed(sim, n=steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc = sim.step_async(n)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / n
        if rc != 0:
            raise RuntimeError(f"batched pic_step returned {pic.STATUS.get(rc, rc)}")
        return ms, sim.step(0)

    # schedule of this mix: a few (tile shape, reordering period) candidates,
    # each with the library's tuning of work-groups per tile and field-solve
    # work-groups, timed over 16 steps; the fastest is timed again below
    sched = []
    for tile, se in SWEEP_SCHEDULES:
        sim = pic.Sim(descs, pic.make_options("fp32", tile=tile, track_ids=False, graph=GRAPH,
                                              tile_split=8, sort_every=se, exchange_frac=EXF,
                                              slack=SLACK))
        for r, t in enumerate(table):
            load_run(sim, r, t)
        sim.step(warmup)
        tuned = sim.tune(2)
        sim.step(8)
        cms, _ = timed(sim, 16)
        sched.append(dict(tile=tile, sort_every=se, tile_split=tuned["tile_split"],
                          cg_blocks=tuned["cg_blocks"], ms_per_step=cms))
        sim.close()
    best = min(sched, key=lambda r: r["ms_per_step"])
    sim = pic.Sim(descs, pic.make_options("fp32", tile=best["tile"], track_ids=False,
                                          graph=GRAPH, tile_split=best["tile_split"],
                                          cg_blocks=best["cg_blocks"],
                                          sort_every=best["sort_every"], exchange_frac=EXF,
                                          slack=SLACK))
    for r, t in enumerate(table):
        load_run(sim, r, t)
    sim.step(warmup + 8)
    tuned = dict(tile_split=best["tile_split"], cg_blocks=best["cg_blocks"])
    ms, st = timed(sim)
    cg_iters = sum(sum(s["iters"]) for s in st)
    sim.close()
    learned = None
    if learned_pairs > 0:
        # the learned aid: one network per distinct (cfl, theta) of the table,
        # trained on the pairs of that operator's first run
        sim = pic.Sim(descs, pic.make_options("fp32", tile=best["tile"], track_ids=False,
                                              graph=GRAPH, tile_split=tuned["tile_split"],
                                              cg_blocks=tuned["cg_blocks"], solver="learned",
                                              precond_slots=learned_pairs,
                                              sort_every=best["sort_every"], exchange_frac=EXF,
                                          slack=SLACK))
        for r, t in enumerate(table):
            load_run(sim, r, t)
        sim.precond_use(False)
        sim.precond_collect(True)
        sim.step(learned_pairs)
        sim.precond_collect(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr = sim.precond_train(learned_epochs, 0.0)
        train_s = time.perf_counter() - t0
        sim.precond_use(True)
        retuned = sim.tune(2, splits=(tuned["tile_split"],))
        sim.step(warmup + 8)
        lms, lst = timed(sim)
        sim.close()
        learned = dict(ms_per_step=lms, particle_steps_per_s=n_part / (lms * 1e-3),
                       networks=tr["networks"], train_seconds=train_s,
                       loss_first=tr["loss_first"], loss_last=tr["loss_last"],
                       cg_blocks=retuned["cg_blocks"],
                       cg_iters_last_step=sum(sum(s["iters"]) for s in lst),
                       fallbacks_last_step=sum(s["fallback"] for s in lst),
                       max_relres=max(max(s["relres"]) for s in lst))
    sim.close()
    seq_ms = 0.0
    # one context per run, same tile shape and reordering period
    opts = pic.make_options("fp32", tile=best["tile"], track_ids=False, graph=GRAPH,
                            sort_every=best["sort_every"], exchange_frac=EXF)
    for r, t in enumerate(table):
        one = pic.Sim([descs[r]], opts)
        load_run(one, 0, t)
        one.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        one.step_async(seq_steps)
        torch.cuda.synchronize()
        seq_ms += (time.perf_counter() - t0) * 1e3 / seq_steps
        one.close()
    return dict(runs=len(table), particles=n_part, ms_per_step=ms, tile=list(best["tile"]),
                sort_every=best["sort_every"], schedules=[dict(r, tile=list(r["tile"]))
                                                          for r in sched],
                tile_split=tuned["tile_split"], cg_blocks=tuned["cg_blocks"],
                particle_steps_per_s=n_part / (ms * 1e-3), cg_iters_last_step=cg_iters,
                sequential_ms_per_step=seq_ms, batched_speedup=seq_ms / ms, learned=learned)


NET_FLOP_PER_CELL = 2 * 9 * (1 * 32 + 32 * 32 + 32 * 1)   # three 3x3 layers, 1->32->32->1
MFMA_BF16_PEAK_TFLOPS = 2500.0


def net_rate(pic, torch, cfg, reps=20):
    """Application rate of the learned network N on one field of the workload
    grid: the BF16 matrix-core form (19,584 FLOP per cell) against the bf16
    dense peak, and the collapsed 7x7 form (98 FLOP per cell)."""
    import ctypes
    run = pic.run_desc(cfg["nx"], cfg["ny"], 0.1, cfg["cfl"], cfg["theta"], cfg["order"],
                       [(-1.0, 1.0, 1), (1.0, 1.0, 1)])
    sim = pic.Sim([run], pic.make_options("fp32", solver="learned", precond_slots=1))
    x = torch.randn(cfg["ny"], cfg["nx"], dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    out = {}
    for name, form in (("mfma", pic.PIC_NET_MFMA), ("collapsed", pic.PIC_NET_COLLAPSED)):
        def call():
            rc = sim.L.pic_precond_apply(sim.ctx, form, cfg["nx"], cfg["ny"],
                                         ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(y.data_ptr()))
            if rc != 0:
                raise RuntimeError("pic_precond_apply failed")
        call()
        t0 = time.perf_counter()
        for _ in range(reps):
            call()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        cells = cfg["nx"] * cfg["ny"]
        flop = (NET_FLOP_PER_CELL if name == "mfma" else 2 * 49) * cells
        out[name] = dict(ms_per_application=ms, tflops=flop / (ms * 1e-3) / 1e12)
    out["mfma"]["frac_of_bf16_peak"] = out["mfma"]["tflops"] / MFMA_BF16_PEAK_TFLOPS
    out["note"] = "one field per call, call includes the library's stream synchronisation"
    sim.close()
    return out


def large_share(pic, torch, steps=10, warmup=300, tile=(16, 32), tile_split=1, pairs=8,
                epochs=50):
    """The large single-GPU share: periodic 8192 x 2048, pair plasma at
    gamma0 = 40, 64 ppc/species (2.1e9 particles), order 3, CFL 1, theta 0.6,
    FP32 particles, loaded on the device, with the learned aid: the first
    `pairs` steps run plain CG (timed, and recorded as training pairs), the
    network is trained, `warmup` untimed steps on the learned solver take the
    run past the saturation of the numerical Cherenkov instability (as in the
    1024 x 256 form), then the timed steps."""
    from synth import loads
    nx, ny, ppc = 8192, 2048, 64
    Q = loads.macro_charge(40.0, 0.1, 0.1, ppc)
    run = pic.run_desc(nx, ny, 0.1, 1.0, 0.6, 3, [(-Q, Q, ppc), (Q, Q, ppc)], cg_rtol=1e-8)
    sim = pic.Sim([run], pic.make_options("fp32", tile=tile, tile_split=tile_split,
                                          track_ids=False, solver="learned",
                                          precond_slots=pairs, sort_every=SORT,
                                          exchange_frac=EXF, slack=SLACK))
    for s in range(2):
        sim.load_plasma(0, s, ppc, 40.0, 0.01, 0)
    n = 2 * nx * ny * ppc
    # plain CG steps, recorded as training pairs
    sim.precond_use(False)
    sim.precond_collect(True)
    sim.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_plain = sim.step(pairs)[0]
    plain_ms = (time.perf_counter() - t0) * 1e3 / pairs
    tim_plain = sim.get_timing()
    sim.timing(False)
    sim.precond_collect(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr = sim.precond_train(epochs, 0.0)
    train_s = time.perf_counter() - t0
    sim.precond_use(True)
    retune = sim.tune(1, splits=(tile_split,))
    if warmup:
        log(f"bench: large share: {warmup} untimed steps")
        sim.step(warmup)
    torch.cuda.synchronize()
    sim.timing(True)
    t0 = time.perf_counter()
    rc = sim.step_async(steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    if rc != 0:
        raise RuntimeError(f"large share pic_step returned {pic.STATUS.get(rc, rc)}")
    tim = sim.get_timing()
    st = sim.step(0)[0]
    push_ms = tim["push"]["ms"] / max(1, tim["push"]["launches"])
    out = dict(workload="periodic 8192x2048, pair gamma0=40, 64 ppc/species, order 3, CFL 1.0, "
                        "theta 0.6 (FP32 particles, learned aid)",
               particles=n, workspace_gb=sim.info.workspace_bytes / 1e9, warmup=warmup,
               ms_per_step=ms,
               particle_steps_per_s=n / (ms * 1e-3), push_ms=push_ms,
               push_achieved_gbs=BYTES_PER_PARTICLE["fp32"] * n / (push_ms * 1e-3) / 1e9,
               field_solve_ms=tim["field_solve"]["ms"] / steps, cg_iters=st["iters"],
               learned_iters=st["learned_iters"], fallback=st["fallback"],
               max_relres=max(st["relres"]), cg_blocks=retune["cg_blocks"],
               training=dict(pairs=pairs, epochs=epochs, seconds=train_s,
                             loss_first=tr["loss_first"], loss_last=tr["loss_last"]),
               plain_cg=dict(ms_per_step=plain_ms, particle_steps_per_s=n / (plain_ms * 1e-3),
                             field_solve_ms=tim_plain["field_solve"]["ms"] / pairs,
                             cg_iters=st_plain["iters"],
                             note=f"the {pairs} collection steps (untuned field-solve grid, "
                                  "pair recording included)"))
    sim.close()
    return out


def shock_share(pic, torch, tile, tile_split, steps=20, warmup=2, pairs=8, epochs=50):
    """The shock workload: 4096 x 512 with conducting walls in x, pair flow at
    gamma0 = 40 towards the reflecting wall at x = 0, 32 ppc/species, order 2,
    CFL 1, theta 0.6, FP32 particles, learned aid (pairs from the first
    steps). Every step first injects the flow entering at x_out (host-generated
    slabs, prepared before the timed region; the injection call copies them to
    the device and is inside the timed region)."""
    from synth import loads
    nx, ny, ppc, g0 = 4096, 512, 32, 40.0
    x_out = nx - pic.PIC_WALL_GAP
    Q = loads.macro_charge(g0, 0.1, 0.1, ppc)
    run = pic.run_desc(nx, ny, 0.1, 1.0, 0.6, 2, [(-Q, Q, ppc), (Q, Q, ppc)], cg_rtol=1e-8,
                       bc="shock")
    sim = pic.Sim([run], pic.make_options("fp32", tile=tile, tile_split=tile_split, slack=1.5,
                                          exchange_frac=EXF, track_ids=False, solver="learned",
                                          precond_slots=pairs, sort_every=SORT))
    for s in range(2):
        sim.load_plasma(0, s, ppc, g0, 0.01, 0, direction=-1, x_cells=x_out)
    total = pairs + warmup + steps
    slabs = [loads.shock_injection(x_out, ny, ppc, g0, 0.01, 0, k, 1.0) for k in range(total)]

    def inject(k):
        for s, d in enumerate(slabs[k]):
            sim.inject_particles(0, s, d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"],
                                 d["uz"])
    sim.precond_use(False)
    sim.precond_collect(True)
    for k in range(pairs):
        inject(k)
        sim.step(1)
    st_plain = sim.step(0)[0]
    sim.precond_collect(False)
    tr = sim.precond_train(epochs, 0.0)
    sim.precond_use(True)
    for k in range(pairs, pairs + warmup):
        inject(k)
        sim.step(1)
    torch.cuda.synchronize()
    sim.timing(True)
    t0 = time.perf_counter()
    for k in range(pairs + warmup, total):
        inject(k)
        rc = sim.step_async(1)
        if rc != 0:
            raise RuntimeError(f"shock pic_step returned {pic.STATUS.get(rc, rc)}")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    tim = sim.get_timing()
    st = sim.step(0)[0]
    d = sim.diag(0)
    n = sum(d["n_particles"][:2])
    sim.close()
    return dict(workload="shock 4096x512 (walls in x, reflection at x=0, injection at x_out), "
                         "pair flow gamma0=40, 32 ppc/species, order 2, CFL 1.0, theta 0.6 "
                         "(FP32 particles, learned aid)",
                particles=n, ms_per_step=ms, particle_steps_per_s=n / (ms * 1e-3),
                push_ms=tim["push"]["ms"] / max(1, tim["push"]["launches"]),
                field_solve_ms=tim["field_solve"]["ms"] / steps,
                cg_iters_plain=st_plain["iters"], learned_iters=st["learned_iters"],
                fallback=st["fallback"], max_relres=max(st["relres"]),
                training=dict(loss_first=tr["loss_first"], loss_last=tr["loss_last"]),
                note="ms_per_step includes the per-step injection call (host slab copied to "
                     "the device)")


def cpu_baseline(cfg, seconds=15.0):
    """The FP64 oracle on a 4-row strip of the same workload (same grid width,
    ppc, order, gamma0), single-threaded; particle-steps/s of whole steps."""
    import oracle
    from synth import loads
    nx, ny = cfg["nx"], 4
    Q = loads.macro_charge(cfg["gamma0"], 0.1, 0.1, cfg["ppc"])
    ld = loads.pair_plasma_cells(nx, ny, cfg["ppc"], cfg["gamma0"], 0.01, seed=0)
    sp = [oracle.Particles(d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"], d["uz"], q, Q)
          for d, q in zip(ld, (-Q, Q))]
    sim = oracle.Sim(nx, ny, 0.1, 0.1, cfg["cfl"], cfg["theta"], cfg["order"], sp)
    n = sum(p.n for p in sp)
    sim.step()
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds or steps < 2:
        sim.step()
        steps += 1
    dt = time.perf_counter() - t0
    return dict(value=n * steps / dt, unit="particle-steps/s", cores=1, kind="oracle",
                sample=f"{nx}x{ny} strip of the workload ({n} particles), {steps} whole "
                       f"steps after 1 warm-up step, 1 thread, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=300,
                    help="untimed steps before the timed ones (also before each autotuner "
                         "candidate): by step 300 the numerical Cherenkov instability of the "
                         "drifting pair plasma has saturated, and the timed steps see the hot, "
                         "bunched state the rest of a 2000-step run spends its steps in")
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--tile", default="16x16")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 form")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cg-blocks", type=int, default=0, help="field-solve work-groups (0 = auto)")
    ap.add_argument("--sweep-cg", default="", help="comma list of cg_blocks to time (FP32 form)")
    ap.add_argument("--tile-split", type=int, default=0, help="work-groups per tile (0 = auto)")
    ap.add_argument("--sweep-tiles", default="",
                    help="comma list of TXxTY:K tile shapes and splits to time (FP32 form)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 48-run batched sweep")
    ap.add_argument("--no-shock", action="store_true",
                    help="skip the 4096x512 shock workload (walls, reflection, injection)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 8192x2048 large single-GPU share (2.1e9 particles)")
    ap.add_argument("--learned-form", default="collapsed", choices=["collapsed", "mfma"],
                    help="inference form of the network in the timed form")
    ap.add_argument("--no-learned", action="store_true",
                    help="time the FP32 form with plain CG only")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the library's autotuner (tile shape, work-groups per tile, "
                         "field-solve work-groups) and use --tile/--tile-split/--cg-blocks")
    ap.add_argument("--no-graph", action="store_true",
                    help="plain launches instead of replaying captured two-step HIP graphs in "
                         "the timed forms")
    ap.add_argument("--sort-every", type=int, default=-1,
                    help="reorder each tile's particles by cell every n steps in the timed "
                         "forms (0 = never); default: picked by the autotuner (0 without it)")
    ap.add_argument("--train-pairs", type=int, default=8)
    ap.add_argument("--train-epochs", type=int, default=50)
    ap.add_argument("--also-mfma", action="store_true",
                    help="also time the FP32 form with the BF16 matrix-core network")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first copy a 512 MiB buffer three times (a plain copy kernel of known "
                         "size, for scaling HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: multi-GPU runs are not part of this build "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1412_2480_amd as pic
    from synth import loads
    global GRAPH, SORT
    GRAPH = not args.no_graph
    SORT = max(0, args.sort_every)

    cfg = CONFIGS[args.config]
    tile = tuple(int(v) for v in args.tile.split("x"))
    if args.calib_copy:
        # A plain elementwise kernel of known size for scaling the HBM traffic
        # counters: the source is written first, then a second 1 GiB buffer is
        # written so the source is no longer resident in the 256 MB Infinity
        # Cache; the multiply then reads 1 GiB and writes 1 GiB.
        n = 256 << 20
        src = torch.full((n,), 1.5, dtype=torch.float32, device="cuda")
        flush = torch.full((n,), 2.5, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst, flush
        log("bench: calibration multiply done (reads 1 GiB, writes 1 GiB)")
    log(f"bench: generating load {cfg['label']}")
    t0 = time.perf_counter()
    load = loads.pair_plasma_cells(cfg["nx"], cfg["ny"], cfg["ppc"], cfg["gamma0"], 0.01, seed=0)
    log(f"bench: load ready in {time.perf_counter() - t0:.1f} s")

    learned = None if args.no_learned else dict(form=args.learned_form, pairs=args.train_pairs,
                                                 epochs=args.train_epochs, lr=1e-3)
    if args.sweep_cg:
        for nb in [int(v) for v in args.sweep_cg.split(",")]:
            for lrn in ([None] if learned is None else [None, learned]):
                r = time_form(pic, torch, cfg, load, "fp32", tile, 10, 2, nb, args.tile_split,
                              lrn)
                log(f"bench: cg_blocks={nb} {'learned' if lrn else 'plain'}: field solve "
                    f"{r['field_solve_ms']:.3f} ms/step, iters {r['cg_iters']}")
    if args.sweep_tiles:
        for item in args.sweep_tiles.split(","):
            shape, k = item.split(":")
            tt = tuple(int(v) for v in shape.split("x"))
            for prec in ("fp32", "fp64"):
                r = time_form(pic, torch, cfg, load, prec, tt, 20, 20, args.cg_blocks, int(k))
                log(f"bench: {prec} tile {shape} split {k}: push {r['push_ms']:.3f} ms, "
                    f"step {r['ms_per_step']:.3f} ms")
    tune = None
    if not args.no_autotune:
        from paper_1412_2480_amd.tune import autotune
        from synth import loads as _l
        Q = _l.macro_charge(cfg["gamma0"], 0.1, 0.1, cfg["ppc"])
        run = pic.run_desc(cfg["nx"], cfg["ny"], 0.1, cfg["cfl"], cfg["theta"], cfg["order"],
                           [(-Q, Q, cfg["ppc"]), (Q, Q, cfg["ppc"])], cg_rtol=1e-8)

        def _load(sim):
            for s_ in range(2):
                d = load[s_]
                sim.load_particles(0, s_, d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"],
                                   d["uz"])
        t0 = time.perf_counter()
        # the shape search runs with reordering on (it changes the ranking);
        # the reordering period is tuned on the chosen shape afterwards
        best, table = autotune([run], _load, dict(precision="fp32", track_ids=False,
                                                  tile_split=8, exchange_frac=EXF, slack=SLACK,
                                                  sort_every=8 if args.sort_every < 0
                                                  else args.sort_every),
                               warmup=args.warmup)
        tune = dict(best={k: best[k] for k in ("tile", "tile_split", "cg_blocks",
                                               "ms_per_step")},
                    table=[{k: r[k] for k in ("tile", "tile_split", "cg_blocks",
                                              "ms_per_step")} for r in table],
                    seconds=time.perf_counter() - t0)
        tile = tuple(best["tile"])
        args.tile_split = best["tile_split"]
        args.cg_blocks = best["cg_blocks"]
        log(f"bench: autotune picked tile {tile} split {args.tile_split} cg_blocks "
            f"{args.cg_blocks} ({tune['seconds']:.1f} s)")
        if args.sort_every < 0:
            from paper_1412_2480_amd.tune import tune_sort_every
            t0 = time.perf_counter()
            SORT, sort_table = tune_sort_every(
                [run], _load, dict(precision="fp32", track_ids=False, tile=tile,
                                   tile_split=args.tile_split, cg_blocks=args.cg_blocks,
                                   exchange_frac=EXF, slack=SLACK),
                candidates=(0, 3, 4, 8, 16), warmup=args.warmup)
            tune["sort_every"] = SORT
            tune["sort_table"] = sort_table
            tune["seconds"] += time.perf_counter() - t0
            log(f"bench: autotune picked sort_every {SORT} " + ", ".join(
                f"{r['sort_every']}: {r['ms_per_step']:.3f} ms" for r in sort_table))
    log("bench: FP32 form" + ("" if learned is None else f" + learned ({args.learned_form})"))
    fast = time_form(pic, torch, cfg, load, "fp32", tile, args.steps, args.warmup, args.cg_blocks,
                     args.tile_split, learned, retune=not args.no_autotune)
    log(f"bench: FP32 {fast['ms_per_step']:.3f} ms/step, field solve "
        f"{fast['field_solve_ms']:.3f} ms, iters {fast['cg_iters']}")
    fast_cg = None
    if learned is not None:
        log("bench: FP32 form, plain CG")
        fast_cg = time_form(pic, torch, cfg, load, "fp32", tile, args.steps, args.warmup,
                            args.cg_blocks, args.tile_split)
        log(f"bench: FP32 plain CG {fast_cg['ms_per_step']:.3f} ms/step, field solve "
            f"{fast_cg['field_solve_ms']:.3f} ms, iters {fast_cg['cg_iters']}")
    mfma = None
    if args.also_mfma and learned is not None and args.learned_form != "mfma":
        log("bench: FP32 form + learned (mfma)")
        mfma = time_form(pic, torch, cfg, load, "fp32", tile, max(10, args.steps // 4),
                         args.warmup, args.cg_blocks, args.tile_split, dict(learned, form="mfma"))
        log(f"bench: FP32 mfma {mfma['ms_per_step']:.3f} ms/step, field solve "
            f"{mfma['field_solve_ms']:.3f} ms, iters {mfma['cg_iters']}")
    plain = None
    if not args.no_fp64:
        # the baseline gets its own schedule: shape search and reordering
        # period tuned for the FP64 form
        t64 = dict(tile=tile, tile_split=args.tile_split, cg_blocks=args.cg_blocks,
                   sort_every=SORT)
        if tune is not None:
            from paper_1412_2480_amd.tune import autotune, tune_sort_every
            b64, _ = autotune([run], _load, dict(precision="fp64", track_ids=False, tile_split=8,
                                                 exchange_frac=EXF, slack=SLACK, sort_every=8),
                              shapes=((4, 32), (8, 32), (16, 32), (16, 16)), warmup=args.warmup)
            k64, _ = tune_sort_every([run], _load, dict(precision="fp64", track_ids=False,
                                                        tile=b64["tile"],
                                                        tile_split=b64["tile_split"],
                                                        cg_blocks=b64["cg_blocks"],
                                                        exchange_frac=EXF, slack=SLACK),
                                     candidates=(0, 4, 8, 16), warmup=args.warmup)
            t64 = dict(tile=tuple(b64["tile"]), tile_split=b64["tile_split"],
                       cg_blocks=b64["cg_blocks"], sort_every=k64)
            tune["fp64_schedule"] = dict(t64, tile=list(t64["tile"]))
            log(f"bench: FP64 schedule: tile {t64['tile']} split {t64['tile_split']} cg_blocks "
                f"{t64['cg_blocks']} sort_every {k64}")
        log("bench: FP64 form")
        plain = time_form(pic, torch, cfg, load, "fp64", t64["tile"], args.steps, args.warmup,
                          t64["cg_blocks"], t64["tile_split"], sort_every=t64["sort_every"])
        log(f"bench: FP64 {plain['ms_per_step']:.3f} ms/step")
    del load

    def run_batched():
        log("bench: batched 48-run sweep")
        b = batched_sweep(pic, torch, 20, 3)
        log(f"bench: batched {b['ms_per_step']:.3f} ms/step for {b['runs']} runs "
            f"(tile {tuple(b['tile'])}, sort_every {b['sort_every']}), "
            f"sequential {b['sequential_ms_per_step']:.3f} ms")
        if b["learned"]:
            bl = b["learned"]
            log(f"bench: batched learned {bl['ms_per_step']:.3f} ms/step "
                f"({bl['networks']} networks, trained in {bl['train_seconds']:.2f} s), "
                f"CG iterations per step {b['cg_iters_last_step']} -> "
                f"{bl['cg_iters_last_step']}")
        return b

    def run_large():
        log("bench: large single-GPU share (8192x2048, 2.1e9 particles)")
        g = large_share(pic, torch, tile=tile, tile_split=max(1, args.tile_split),
                        warmup=args.warmup)
        log(f"bench: large share {g['ms_per_step']:.1f} ms/step, push "
            f"{g['push_ms']:.1f} ms ({g['push_achieved_gbs']:.0f} GB/s), field solve "
            f"{g['field_solve_ms']:.1f} ms learned vs "
            f"{g['plain_cg']['field_solve_ms']:.1f} ms plain CG, trained in "
            f"{g['training']['seconds']:.2f} s")
        return g

    def run_shock():
        log("bench: shock workload (4096x512, walls, injection)")
        k = shock_share(pic, torch, tile, max(1, args.tile_split))
        log(f"bench: shock {k['ms_per_step']:.2f} ms/step ({k['particles']:.3g} "
            f"particles), push {k['push_ms']:.2f} ms, field solve "
            f"{k['field_solve_ms']:.2f} ms, CG iterations {k['cg_iters_plain']} -> "
            f"{k['learned_iters']}")
        return k

    def run_net():
        r = net_rate(pic, torch, cfg)
        log(f"bench: network application: mfma {r['mfma']['ms_per_application']:.3f} ms "
            f"({r['mfma']['tflops']:.1f} TFLOP/s), collapsed "
            f"{r['collapsed']['ms_per_application']:.3f} ms")
        return r

    def run_cpu():
        log("bench: oracle CPU baseline")
        return cpu_baseline(cfg, args.cpu_seconds)

    batched = None if args.no_batched else run_leg("batched sweep", run_batched)
    large = None if args.no_large else run_leg("large share", run_large)
    shock = None if args.no_shock else run_leg("shock workload", run_shock)
    net = None if args.no_learned else run_leg("network rate", run_net)
    cpu = None if args.no_cpu else run_leg("CPU baseline", run_cpu)

    n_part = fast["n_particles"]
    achieved = BYTES_PER_PARTICLE["fp32"] * n_part / (fast["push_ms"] * 1e-3) / 1e9
    traffic, traffic_src = measured_traffic("fp32", tile, args.tile_split, cfg["order"], n_part,
                                            SORT, args.warmup)
    def solve_info(r):
        return None if r is None else dict(
            ms_per_step=r["ms_per_step"], particle_steps_per_s=r["particle_steps_per_s"],
            field_solve_ms_per_step=r["field_solve_ms"], cg_iters_last_step=r["cg_iters"],
            learned_iters_last_step=r["learned_iters"], fallback=r["fallback"],
            relres_last_step=r["relres"], training=r["train"])

    line = {
        "metric": "particle-steps/s + field-solve ms/step; FP32+learned vs plain FP64, same GPU",
        "value": fast["particle_steps_per_s"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fast["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 particles, f64 fields/CG" + ("" if learned is None else
                                                    f", learned aid ({args.learned_form})"),
        "data": "synthetic (seeded Maxwell-Juettner pair plasma)",
        "config": {"workload": cfg["label"], "particles": n_part, "cells": cfg["nx"] * cfg["ny"],
                   "tile": list(tile), "sort_every": SORT, "graph": GRAPH, "cg_rtol": 1e-8},
        "field_solve_ms_per_step": fast["field_solve_ms"],
        "cg_iters_last_step": fast["cg_iters"],
        "learned": solve_info(fast) if learned is not None else None,
        "fp32_plain_cg": solve_info(fast_cg),
        "fp32_learned_mfma": solve_info(mfma),
        "breakdown_ms": {k: fast[k] for k in ("push_ms", "rebin_ms", "current_sum_ms",
                                              "sort_ms_per_step", "field_solve_ms")},
        "plain_fp64": None if plain is None else {
            "particle_steps_per_s": plain["particle_steps_per_s"],
            "ms_per_step": plain["ms_per_step"],
            "field_solve_ms_per_step": plain["field_solve_ms"],
            "push_ms": plain["push_ms"],
            "cg_iters_last_step": plain["cg_iters"],
            "speedup_of_timed_form": plain["ms_per_step"] / fast["ms_per_step"],
            "field_solve_speedup_of_timed_form": plain["field_solve_ms"] / fast["field_solve_ms"],
            "schedule": None if tune is None else tune.get("fp64_schedule"),
        },
        "roofline": {"bound": "hbm", "kernel": "fused particle push (gather+Boris+move+deposit)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "bytes per launch", "traffic_source": traffic_src,
                     "bytes_per_particle_step": BYTES_PER_PARTICLE["fp32"],
                     "algorithmic_bytes_per_launch": BYTES_PER_PARTICLE["fp32"] * n_part,
                     "avg_launch_ms": fast["push_ms"], "tile": list(tile),
                     "tile_split": args.tile_split, "sort_every": SORT},
        "autotune": tune,
        "learned_net": net,
        "large_share": large,
        "shock": shock,
        "batched_sweep": batched,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
