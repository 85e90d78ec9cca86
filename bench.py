#!/usr/bin/env python3
"""Throughput of the PIC hot path on one MI355X.

Headline workload (the largest single-GPU configuration): periodic
8192 x 2048 grid, dx = 0.1 c/omega_pe, pair plasma at gamma0 = 40 with
T = 0.01 m c^2, 64 particles/cell/species (2^31 = 2,147,483,648 particles,
FP32 SoA, loaded on the device from the seeded generator), cubic (order-3)
shape, CFL 1.0, theta = 0.6, field CG to 1e-8, FP32 particles with the
learned CG aid. One step = gather + Boris push + move + Esirkepov deposit of
every particle, tile re-binning, the current reduction and the implicit
field solve (RHS of Eq. (7), learned PCG, update of Eqs. (5)-(6)).

The network is trained on the (b, dB) pairs of the first steps, solved by
plain CG (those steps also give the plain-CG field-solve time); training is a
one-time set-up, timed and reported on its own and folded into a whole-run
figure. Then --warmup untimed steps and --steps timed steps; the particle
kernel's launches inside the timed region are timed with HIP events on the
context's stream (the roofline's achieved bandwidth). The same workload is
then taken on, untimed, for --later-after more steps and timed again: the
state in which a long run spends most of its steps (the beam has spread and
the density has bunched, which costs the particle kernel LDS conflicts).

Further legs: the 1024 x 256 single run (FP32 + learned, FP32 with plain CG,
and the plain FP64 form on a schedule tuned for it: the FP32-vs-FP64 factor
on the same GPU), the 48-run sweep in one context, the shock workload
(walls, device injection), the explicit FDTD variant against the implicit
scheme, the network's application rate, and the FP64 CPU oracle on a strip of
the headline workload (one thread and all threads).

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

HEADLINE = dict(nx=8192, ny=2048, ppc=64, gamma0=40.0, order=3, cfl=1.0, theta=0.6,
                label="periodic 8192x2048, pair gamma0=40, 64 ppc/species (2^31 particles), "
                      "order 3, CFL 1.0, theta 0.6")
# schedule of the headline workload, measured on it (particle kernel, current
# reduction and reordering per step at the cold start): 2x64 tiles, one
# work-group per tile, reordering every 4 steps 65.3 ms; 2x64 with two
# work-groups 70.6; 4x32 with two 80.6; 4x64 78.7; 2x128 96.0
HEADLINE_TILE, HEADLINE_SPLIT, HEADLINE_SORT = (2, 64), 1, 4

CONFIGS = {
    # name: nx, ny, ppc, gamma0, order, cfl, theta
    "1024x256": dict(nx=1024, ny=256, ppc=64, gamma0=40.0, order=3, cfl=1.0, theta=0.6,
                     label="periodic 1024x256, pair gamma0=40, 64 ppc/species, order 3, "
                           "CFL 1.0, theta 0.6"),
    "64x64": dict(nx=64, ny=64, ppc=16, gamma0=20.0, order=1, cfl=1.0, theta=0.6,
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
        # the warm-up length counts: the spread, bunched plasma of a long run
        # moves other bytes than the cold start
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
        return rec, os.path.relpath(path, ROOT)
    return None, None


# issue ceiling of the vector ALU: a wave64 instruction occupies a 16-lane
# SIMD for 4 cycles; 256 CUs x 4 SIMDs at 2.4 GHz (packed FP32 is not used)
VALU_CYCLES_PER_INST, N_SIMD, CLOCK_HZ = 4, 1024, 2.4e9


def ceilings(rec, n_particles, launch_ms):
    """The particle kernel against its issue and LDS ceilings, from the
    instruction counts of the counter record (which are fixed by the kernel's
    code and the particle count) and the live launch time."""
    if rec is None or "valu_instructions_per_wavefront_of_64_particles" not in rec:
        return None
    vpw = rec["valu_instructions_per_wavefront_of_64_particles"]
    valu_ms = n_particles / 64 * vpw * VALU_CYCLES_PER_INST / (N_SIMD * CLOCK_HZ) * 1e3
    return {"valu_issue": {"ms": valu_ms, "frac": valu_ms / launch_ms,
                           "instructions_per_wavefront": vpw},
            "lds": {"active_fraction_counted": rec["lds_active_fraction"],
                    "instructions_per_wavefront": rec["lds_instructions_per_wavefront_of_64_particles"]},
            "note": "VALU: the counted instructions at one wave64 instruction per SIMD every 4 "
                    "cycles; LDS: cycles with the LDS pipe active over the kernel's cycles "
                    "(SQ_LDS_IDX_ACTIVE per CU / SQ_BUSY_CYCLES per shader engine), counted "
                    "on the same launches as the traffic"}


GRAPH = True    # pic_step replays captured two-step HIP graphs (--no-graph: plain launches)
SORT = 0        # pic_options.sort_every of the timed forms (autotuned, or --sort-every)
# (tile shape, reordering period) candidates of the 48-run sweep
SWEEP_SCHEDULES = (((16, 16), 0), ((4, 32), 8), ((8, 16), 8), ((2, 32), 8))
SLACK = 0.5     # tile slots over ppc*cells: the densities of the drifting plasma bunch
                # over a long run; with the staggered gather (where the numerical
                # Cherenkov instability grows at CFL 1) a tile of the default 0.25
                # overflowed within the 2000-step run


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
                                          slack=SLACK))
    for s in range(2):
        d = load[s]
        sim.load_particles(0, s, d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"], d["uz"])
    return sim


def time_form(pic, torch, cfg, load, precision, tile, steps, warmup, cg_blocks=0, tile_split=0,
              learned=None, retune=False, sort_every=None):
    """learned: None (plain CG) or dict(form, pairs, epochs, lr): collect that
    many pairs with plain CG in the first steps, train, then take the learned
    path for the warm-up and the timed steps (as a run would: the network
    trained on the first steps' pairs keeps 3 iterations per component over a
    long run)."""
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
                                              tile_split=8, sort_every=se,
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
                                          sort_every=best["sort_every"],
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
                                              sort_every=best["sort_every"],
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
                            sort_every=best["sort_every"])
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


def net_rate(pic, torch, cfg, reps=10):
    """Application rate of the learned network N on one field of the headline
    grid (16.8M cells): the BF16 matrix-core form (19,584 FLOP per cell)
    against the bf16 dense peak, and the collapsed 7x7 form (98 FLOP per
    cell). Timed with HIP events on the context's stream around the calls (a
    call ends with the library's stream synchronisation, a few microseconds
    against milliseconds of kernel time at this size)."""
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
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(sim.stream)
        for _ in range(reps):
            call()
        ev1.record(sim.stream)
        ev1.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        cells = cfg["nx"] * cfg["ny"]
        flop = (NET_FLOP_PER_CELL if name == "mfma" else 2 * 49) * cells
        out[name] = dict(ms_per_application=ms, tflops=flop / (ms * 1e-3) / 1e12)
    out["mfma"]["frac_of_bf16_peak"] = out["mfma"]["tflops"] / MFMA_BF16_PEAK_TFLOPS
    out["grid"] = [cfg["nx"], cfg["ny"]]
    out["note"] = "one field per call, HIP events on the context stream"
    sim.close()
    return out


def headline(pic, torch, steps, warmup, later_after=300, pairs=8, epochs=50):
    """The headline workload (HEADLINE dict): 2^31 particles loaded on the device,
    FP32 particles with the learned aid. Returns the timed figures: wall
    clock over `steps` steps after `warmup` untimed ones, the particle
    kernel's average launch time from HIP events on the context stream over
    the same launches, the field solve, and (if later_after > 0) the
    same after that many further untimed steps."""
    from synth import loads
    c = HEADLINE
    nx, ny, ppc = c["nx"], c["ny"], c["ppc"]
    Q = loads.macro_charge(c["gamma0"], 0.1, 0.1, ppc)
    run = pic.run_desc(nx, ny, 0.1, c["cfl"], c["theta"], c["order"], [(-Q, Q, ppc), (Q, Q, ppc)],
                       cg_rtol=1e-8, cg_maxit=200)
    sim = pic.Sim([run], pic.make_options("fp32", tile=HEADLINE_TILE, tile_split=HEADLINE_SPLIT,
                                          track_ids=False, solver="learned",
                                          precond_slots=pairs, sort_every=HEADLINE_SORT, slack=SLACK))
    t0 = time.perf_counter()
    for s in range(2):
        sim.load_plasma(0, s, ppc, c["gamma0"], 0.01, 0)
    torch.cuda.synchronize()
    load_s = time.perf_counter() - t0
    n = 2 * nx * ny * ppc
    # the first steps: plain CG, recorded as training pairs
    sim.precond_use(False)
    sim.precond_collect(True)
    sim.timing(True)
    t0 = time.perf_counter()
    st_plain = sim.step(pairs)[0]
    plain_s = time.perf_counter() - t0
    tim_plain = sim.get_timing()
    sim.timing(False)
    sim.precond_collect(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr = sim.precond_train(epochs, 0.0)
    train_s = time.perf_counter() - t0
    sim.precond_use(True)
    t0 = time.perf_counter()
    retune = sim.tune(1, splits=(HEADLINE_SPLIT,))
    tune_s = time.perf_counter() - t0

    def timed(k):
        torch.cuda.synchronize()
        sim.timing(True)
        t0 = time.perf_counter()
        rc = sim.step_async(k)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / k
        if rc != 0:
            raise RuntimeError(f"headline pic_step returned {pic.STATUS.get(rc, rc)}")
        tim = sim.get_timing()
        sim.timing(False)
        st = sim.step(0)[0]
        push = tim["push"]
        return dict(ms_per_step=ms, particle_steps_per_s=n / (ms * 1e-3),
                    push_ms=push["ms"] / max(1, push["launches"]), push_launches=push["launches"],
                    field_solve_ms=tim["field_solve"]["ms"] / k,
                    rebin_ms=tim["rebin"]["ms"] / k, current_sum_ms=tim["current_sum"]["ms"] / k,
                    sort_ms_per_step=tim["sort"]["ms"] / k, cg_iters=st["iters"],
                    learned_iters=st["learned_iters"], fallback=st["fallback"],
                    max_relres=max(st["relres"]))

    if warmup:
        sim.step(warmup)
    main_t = timed(steps)
    sat = None
    if later_after > 0:
        log(f"bench: headline: {later_after} more untimed steps (later phase)")
        sim.step(later_after)
        sat = dict(timed(min(steps, 10)), after_steps=pairs + warmup + steps + later_after)
    d = sim.diag(0)
    out = dict(workload=c["label"] + " (FP32 particles, learned aid)", particles=n,
               workspace_gb=sim.info.workspace_bytes / 1e9, load_seconds=load_s,
               tile=list(HEADLINE_TILE), tile_split=HEADLINE_SPLIT, sort_every=HEADLINE_SORT,
               cg_blocks=retune["cg_blocks"], timed=main_t, later=sat,
               training=dict(pairs=pairs, epochs=epochs, seconds=train_s, tune_seconds=tune_s,
                             loss_first=tr["loss_first"], loss_last=tr["loss_last"]),
               plain_cg=dict(ms_per_step=plain_s * 1e3 / pairs,
                             field_solve_ms=tim_plain["field_solve"]["ms"] / pairs,
                             cg_iters=st_plain["iters"],
                             note=f"the first {pairs} steps (plain CG, pairs recorded)"),
               gauss_max=d["gauss_max"], n_particles=d["n_particles"][:2])
    # a 1000-step run (the workload's length): collection steps, training,
    # then the steps up to the later measurement at the timed rate and the
    # rest at the later rate
    if sat is not None:
        n_cold = sat["after_steps"] - pairs
        run_s = plain_s + train_s + tune_s + (n_cold * main_t["ms_per_step"] + (
            1000 - sat["after_steps"]) * sat["ms_per_step"]) * 1e-3
        note = (f"the {pairs} collection steps, training, tuning, {n_cold} steps at the timed "
                f"rate and {1000 - sat['after_steps']} at the later-phase rate")
    else:
        run_s = plain_s + train_s + tune_s + (1000 - pairs) * main_t["ms_per_step"] * 1e-3
        note = (f"the {pairs} collection steps, training, tuning and {1000 - pairs} steps at "
                "the timed rate (later phase not measured)")
    out["whole_run_1000_steps"] = dict(seconds=run_s, ms_per_step=run_s * 1e3 / 1000,
                                       particle_steps_per_s=n * 1000 / run_s, note=note)
    sim.close()
    return out


def shock_share(pic, torch, tile, tile_split, steps=20, warmup=5, pairs=8, epochs=50):
    """The shock workload: 4096 x 512 with conducting walls in x, pair flow at
    gamma0 = 40 towards the reflecting wall at x = 0, 32 ppc/species, order 2,
    CFL 1, theta 0.6, FP32 particles, learned aid (pairs from the first
    steps); the flow entering at x_out is generated on the device before every
    step (pic_set_inflow), inside the timed region, and the steps replay
    captured graphs. Also times the same steps with plain CG."""
    from synth import loads
    nx, ny, ppc, g0 = 4096, 512, 32, 40.0
    x_out = nx - pic.PIC_WALL_GAP
    Q = loads.macro_charge(g0, 0.1, 0.1, ppc)
    run = pic.run_desc(nx, ny, 0.1, 1.0, 0.6, 2, [(-Q, Q, ppc), (Q, Q, ppc)], cg_rtol=1e-8,
                       bc="shock")
    sim = pic.Sim([run], pic.make_options("fp32", tile=tile, tile_split=tile_split, slack=1.5, track_ids=False, solver="learned",
                                          precond_slots=pairs, sort_every=4, graph=GRAPH))
    for s in range(2):
        sim.load_plasma(0, s, ppc, g0, 0.01, 0, direction=-1, x_cells=x_out)
    sim.set_inflow(0, ppc, g0, 0.01, 0)
    sim.precond_use(False)
    sim.precond_collect(True)
    sim.timing(True)
    sim.step(pairs)
    tim_plain = sim.get_timing()
    sim.timing(False)
    st_plain = sim.step(0)[0]
    sim.precond_collect(False)
    tr = sim.precond_train(epochs, 0.0)
    sim.precond_use(True)
    sim.step(warmup)

    def timed():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc = sim.step_async(steps)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        if rc != 0:
            raise RuntimeError(f"shock pic_step returned {pic.STATUS.get(rc, rc)}")
        sim.timing(True)
        sim.step(4)
        tim = sim.get_timing()
        sim.timing(False)
        return ms, tim
    ms, tim = timed()
    st = sim.step(0)[0]
    d = sim.diag(0)
    n = sum(d["n_particles"][:2])
    out = dict(workload="shock 4096x512 (walls in x, reflection at x=0, device inflow at x_out), "
                        "pair flow gamma0=40, 32 ppc/species, order 2, CFL 1.0, theta 0.6 "
                        "(FP32 particles, learned aid)",
               particles=n, ms_per_step=ms, particle_steps_per_s=n / (ms * 1e-3),
               push_ms=tim["push"]["ms"] / max(1, tim["push"]["launches"]),
               field_solve_ms=tim["field_solve"]["ms"] / 4,
               field_solve_ms_plain_cg=tim_plain["field_solve"]["ms"] / pairs,
               cg_iters_plain=st_plain["iters"], learned_iters=st["learned_iters"],
               fallback=st["fallback"], max_relres=max(st["relres"]),
               training=dict(pairs=pairs, loss_first=tr["loss_first"],
                             loss_last=tr["loss_last"]),
               note="ms_per_step includes the device injection of the entering flow")
    sim.precond_use(False)
    ms_cg, tim_cg = timed()
    out["plain_cg"] = dict(ms_per_step=ms_cg, field_solve_ms=tim_cg["field_solve"]["ms"] / 4,
                           cg_iters=sim.step(0)[0]["iters"])
    sim.close()
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, seconds=10.0, rows=4):
    """The FP64 oracle (plain C with OpenMP) on a strip of the headline
    workload: the full width, `rows` rows, the same ppc, order, gamma0, CFL
    and theta; particle-steps/s of whole steps, on one thread and on all the
    host's threads (about `seconds` of CPU work each)."""
    import oracle
    from synth import loads
    nx, ny = cfg["nx"], rows
    Q = loads.macro_charge(cfg["gamma0"], 0.1, 0.1, cfg["ppc"])
    ld = loads.pair_plasma_cells(nx, ny, cfg["ppc"], cfg["gamma0"], 0.01, seed=0)
    nproc = os.cpu_count() or 1
    out = {}
    for threads in (1, nproc):
        oracle.set_threads(threads)
        sp = [oracle.Particles(d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"], d["uz"],
                               q, Q) for d, q in zip(ld, (-Q, Q))]
        sim = oracle.Sim(nx, ny, 0.1, 0.1, cfg["cfl"], cfg["theta"], cfg["order"], sp)
        n = sum(p.n for p in sp)
        sim.step()
        steps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < seconds or steps < 2:
            sim.step()
            steps += 1
        dt = time.perf_counter() - t0
        out[threads] = dict(value=n * steps / dt, steps=steps, seconds=dt, particles=n)
    oracle.set_threads(0)
    best = out[nproc]
    return dict(value=best["value"], unit="particle-steps/s", cores=nproc, kind="oracle",
                sample=f"{nx}x{ny} strip of the headline workload ({best['particles']} "
                       f"particles), {best['steps']} whole steps after 1 warm-up step on "
                       f"{nproc} threads ({best['seconds']:.1f} s); a per-particle-step rate "
                       "extrapolated to the full grid",
                one_thread=dict(value=out[1]["value"], steps=out[1]["steps"],
                                seconds=out[1]["seconds"]),
                nproc=nproc, cpu_model=_cpu_model())


def single_run_legs(pic, torch, args, learned):
    """The 1024 x 256 single run: FP32 + learned, FP32 with plain CG and the
    plain FP64 form, each on its own tuned schedule; returns the three
    timings, the tuning tables and the FP32/FP64 factor."""
    from synth import loads
    global SORT
    cfg = CONFIGS["1024x256"]
    log(f"bench: generating load {cfg['label']}")
    load = loads.pair_plasma_cells(cfg["nx"], cfg["ny"], cfg["ppc"], cfg["gamma0"], 0.01, seed=0)
    tile = (4, 32)
    split, cgb = 2, 128
    Q = loads.macro_charge(cfg["gamma0"], 0.1, 0.1, cfg["ppc"])
    run = pic.run_desc(cfg["nx"], cfg["ny"], 0.1, cfg["cfl"], cfg["theta"], cfg["order"],
                       [(-Q, Q, cfg["ppc"]), (Q, Q, cfg["ppc"])], cg_rtol=1e-8)

    def _load(sim):
        for s_ in range(2):
            d = load[s_]
            sim.load_particles(0, s_, d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"], d["uz"])
    tune = None
    if not args.no_autotune:
        from paper_1412_2480_amd.tune import autotune, tune_sort_every
        t0 = time.perf_counter()
        best, table = autotune([run], _load, dict(precision="fp32", track_ids=False,
                                                  tile_split=8, slack=SLACK,
                                                  sort_every=8), warmup=args.warmup)
        tile, split, cgb = tuple(best["tile"]), best["tile_split"], best["cg_blocks"]
        SORT, sort_table = tune_sort_every(
            [run], _load, dict(precision="fp32", track_ids=False, tile=tile, tile_split=split,
                               cg_blocks=cgb, slack=SLACK),
            candidates=(0, 3, 4, 8), warmup=args.warmup)
        tune = dict(best=dict(tile=list(tile), tile_split=split, cg_blocks=cgb,
                              sort_every=SORT),
                    table=[{k: r[k] for k in ("tile", "tile_split", "cg_blocks", "ms_per_step")}
                           for r in table], sort_table=sort_table,
                    seconds=time.perf_counter() - t0)
        log(f"bench: 1024x256 autotune: tile {tile} split {split} cg_blocks {cgb} sort_every {SORT}")
    else:
        SORT = 4
    fast = time_form(pic, torch, cfg, load, "fp32", tile, args.steps, args.warmup, cgb, split,
                     learned, retune=not args.no_autotune)
    log(f"bench: 1024x256 FP32 + learned {fast['ms_per_step']:.3f} ms/step, push {fast['push_ms']:.3f}, "
        f"field solve {fast['field_solve_ms']:.3f} ms, iters {fast['cg_iters']}")
    fast_cg = time_form(pic, torch, cfg, load, "fp32", tile, args.steps, args.warmup, cgb, split)
    log(f"bench: 1024x256 FP32 plain CG {fast_cg['ms_per_step']:.3f} ms/step, field solve "
        f"{fast_cg['field_solve_ms']:.3f} ms, iters {fast_cg['cg_iters']}")
    mfma = None
    if not args.no_mfma and learned is not None:
        mfma = time_form(pic, torch, cfg, load, "fp32", tile, args.steps, args.warmup, cgb, split,
                         dict(learned, form="mfma"))
        log(f"bench: 1024x256 FP32 + learned (mfma) {mfma['ms_per_step']:.3f} ms/step, field solve "
            f"{mfma['field_solve_ms']:.3f} ms")
    plain = None
    if not args.no_fp64:
        t64 = dict(tile=tile, tile_split=1, cg_blocks=256, sort_every=0)
        if tune is not None:
            from paper_1412_2480_amd.tune import autotune, tune_sort_every
            b64, _ = autotune([run], _load, dict(precision="fp64", track_ids=False, tile_split=8, slack=SLACK, sort_every=8),
                              shapes=((2, 64), (4, 32), (8, 32), (16, 16)),
                              warmup=args.warmup)
            k64, _ = tune_sort_every([run], _load, dict(precision="fp64", track_ids=False,
                                                        tile=b64["tile"],
                                                        tile_split=b64["tile_split"],
                                                        cg_blocks=b64["cg_blocks"], slack=SLACK),
                                     candidates=(0, 4, 8), warmup=args.warmup)
            t64 = dict(tile=tuple(b64["tile"]), tile_split=b64["tile_split"],
                       cg_blocks=b64["cg_blocks"], sort_every=k64)
            tune["fp64_schedule"] = dict(t64, tile=list(t64["tile"]))
        plain = time_form(pic, torch, cfg, load, "fp64", t64["tile"], args.steps, args.warmup,
                          t64["cg_blocks"], t64["tile_split"], sort_every=t64["sort_every"])
        log(f"bench: 1024x256 FP64 {plain['ms_per_step']:.3f} ms/step, field solve "
            f"{plain['field_solve_ms']:.3f} ms")
    del load

    def info(r):
        return None if r is None else dict(
            ms_per_step=r["ms_per_step"], particle_steps_per_s=r["particle_steps_per_s"],
            push_ms=r["push_ms"], field_solve_ms_per_step=r["field_solve_ms"],
            cg_iters_last_step=r["cg_iters"], learned_iters_last_step=r["learned_iters"],
            fallback=r["fallback"], relres_last_step=r["relres"], training=r["train"])
    out = dict(workload=cfg["label"], particles=fast["n_particles"], tile=list(tile),
               tile_split=split, sort_every=SORT, fp32_learned=info(fast),
               fp32_plain_cg=info(fast_cg), fp32_learned_mfma=info(mfma), plain_fp64=info(plain),
               breakdown_ms={k: fast[k] for k in ("push_ms", "rebin_ms", "current_sum_ms",
                                                  "sort_ms_per_step", "field_solve_ms")},
               autotune=tune)
    if plain is not None:
        out["speedup_fp32_learned_vs_fp64"] = plain["ms_per_step"] / fast["ms_per_step"]
        out["field_solve_speedup_vs_fp64"] = plain["field_solve_ms"] / fast["field_solve_ms"]
    return out


def explicit_vs_implicit(pic, torch, steps=20, warmup=5):
    """The explicit Yee FDTD variant (Eqs. (3)-(4)) at its stable CFL 0.5
    against the implicit scheme at CFL 1.0 on the 1024 x 256 workload (FP32
    particles): time per step and per unit of simulated time."""
    cfg = CONFIGS["1024x256"]
    from synth import loads
    out = {}
    for scheme, cfl in (("explicit", 0.5), ("implicit", 1.0)):
        Q = loads.macro_charge(cfg["gamma0"], 0.1, 0.1, cfg["ppc"])
        run = pic.run_desc(cfg["nx"], cfg["ny"], 0.1, cfl, 0.6, cfg["order"],
                           [(-Q, Q, cfg["ppc"]), (Q, Q, cfg["ppc"])], cg_rtol=1e-8)
        sim = pic.Sim([run], pic.make_options("fp32", tile=(2, 64), tile_split=2, sort_every=4,
                                              track_ids=False, slack=SLACK,
                                              scheme=scheme, graph=GRAPH))
        for s in range(2):
            sim.load_plasma(0, s, cfg["ppc"], cfg["gamma0"], 0.01, 0)
        sim.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc = sim.step_async(steps)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        if rc != 0:
            raise RuntimeError(f"{scheme} pic_step returned {pic.STATUS.get(rc, rc)}")
        sim.timing(True)
        sim.step(5)
        tim = sim.get_timing()
        sim.close()
        out[scheme] = dict(cfl=cfl, ms_per_step=ms, ms_per_unit_time=ms / (cfl * 0.1),
                           field_ms=tim["field_solve"]["ms"] / 5)
    out["note"] = ("time per step and per 1/omega_pe of simulated time (dt = cfl dx); the "
                   "explicit scheme is stable only for cfl^2 (1 + dx^2/dy^2) <= 1")
    return out


def nci_scans(pic, torch, t_cfl=400.0, t_theta=5000.0):
    """The paper's scans of Sec. 3 (Gamma = 100, 128 x 128, 100 ppc/species,
    cell = Debye length) as batched runs: CFL 0.4 ... 1.0 x orders 1, 2 at
    theta = 0.501 to t = t_cfl dx/c, and theta 0.5 ... 0.503 x orders 1, 2 at
    sigma = 1 to t = t_theta dx/c; growth rates of W_B and the time each scan
    took on the GPU."""
    from paper_1412_2480_amd import nci
    out = {}
    for name, fn, kw in (("cfl", nci.cfl_scan, dict(t_end=t_cfl)),
                         ("theta", nci.theta_scan, dict(t_end=t_theta))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fn(pic, **kw)
        sec = time.perf_counter() - t0
        rows = []
        for r in res:
            c, g = r["case"], r["growth"]
            rows.append(dict(cfl=c["cfl"], theta=c["theta"], order=c["order"],
                             growth_rate_per_dx_over_c=None if g is None else g["rate"],
                             fit_window=None if g is None else [g["t0"], g["t1"]],
                             W_B_max=float(r["W_B"].max()), energy_drift=r["energy_drift"]))
        n_part = sum(2 * r["case"]["n"] ** 2 * r["case"]["ppc"] for r in res)
        steps = int(res[0]["t"].size)
        out[name] = dict(runs=len(res), particles=n_part, steps=steps, seconds=sec,
                         particle_steps_per_s=n_part * steps / sec, rows=rows)
        log(f"bench: NCI {name} scan: {len(res)} runs, {steps} steps in {sec:.1f} s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--later-after", type=int, default=300,
                    help="untimed headline steps before the later-phase timing (0 = skip): "
                         "the state a long run spends most steps in")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline workload (for profiling runs)")
    ap.add_argument("--no-1024", action="store_true", help="skip the 1024x256 legs")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 form")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-batched", action="store_true", help="skip the 48-run batched sweep")
    ap.add_argument("--no-shock", action="store_true", help="skip the shock workload")
    ap.add_argument("--no-explicit", action="store_true",
                    help="skip the explicit-vs-implicit scheme leg")
    ap.add_argument("--no-nci", action="store_true",
                    help="skip the paper's numerical-Cherenkov scans (Sec. 3)")
    ap.add_argument("--learned-form", default="collapsed", choices=["collapsed", "mfma"])
    ap.add_argument("--no-mfma", action="store_true",
                    help="skip the 1024x256 leg with the network applied on the matrix cores")
    ap.add_argument("--no-autotune", action="store_true",
                    help="fixed schedules for the 1024x256 legs instead of the autotuner")
    ap.add_argument("--no-graph", action="store_true",
                    help="plain launches instead of captured two-step HIP graphs (1024x256 legs)")
    ap.add_argument("--train-pairs", type=int, default=8)
    ap.add_argument("--train-epochs", type=int, default=50)
    ap.add_argument("--calib-copy", action="store_true",
                    help="first a plain multiply of a 1 GiB buffer (a copy kernel of known "
                         "size, for scaling HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path has no multi-GPU form "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1412_2480_amd as pic
    global GRAPH
    GRAPH = not args.no_graph
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

    learned = dict(form=args.learned_form, pairs=args.train_pairs, epochs=args.train_epochs,
                   lr=1e-3)
    log(f"bench: headline {HEADLINE['label']}")
    h = headline(pic, torch, args.steps, args.warmup,
                 0 if args.headline_only else args.later_after, args.train_pairs,
                 args.train_epochs)
    t = h["timed"]
    log(f"bench: headline {t['ms_per_step']:.2f} ms/step ({t['particle_steps_per_s']:.3g} "
        f"particle-steps/s), push {t['push_ms']:.2f} ms, field solve {t['field_solve_ms']:.2f} ms "
        f"(plain CG {h['plain_cg']['field_solve_ms']:.2f} ms)")
    if h["later"]:
        sa = h["later"]
        log(f"bench: headline later phase {sa['ms_per_step']:.2f} ms/step, push "
            f"{sa['push_ms']:.2f} ms")
    gc.collect()
    torch.cuda.empty_cache()

    legs = {}
    if not args.headline_only:
        if not args.no_1024:
            legs["single_run_1024x256"] = run_leg("1024x256 legs", lambda: single_run_legs(pic, torch, args, learned))
        if not args.no_explicit:
            legs["explicit_vs_implicit"] = run_leg("explicit scheme",
                                                   lambda: explicit_vs_implicit(pic, torch))
        if not args.no_batched:
            legs["batched_sweep"] = run_leg("batched sweep",
                                            lambda: batched_sweep(pic, torch, 20, 3))
        if not args.no_shock:
            legs["shock"] = run_leg("shock workload",
                                    lambda: shock_share(pic, torch, (4, 32), 2))
        legs["learned_net"] = run_leg("network rate", lambda: net_rate(pic, torch, HEADLINE))
        if not args.no_nci:
            legs["nci_scans"] = run_leg("NCI scans", lambda: nci_scans(pic, torch))
    cpu = None
    if not args.no_cpu and not args.headline_only:
        log("bench: oracle CPU baseline")
        cpu = run_leg("CPU baseline", lambda: cpu_baseline(HEADLINE, args.cpu_seconds))

    n_part = h["particles"]
    alg = BYTES_PER_PARTICLE["fp32"] * n_part
    achieved = alg / (t["push_ms"] * 1e-3) / 1e9
    rec, traffic_src = measured_traffic("fp32", HEADLINE_TILE, HEADLINE_SPLIT, HEADLINE["order"], n_part,
                                        HEADLINE_SORT, args.warmup)
    traffic = None if rec is None else rec["traffic_bytes"]
    line = {
        "metric": "particle-steps/s + field-solve ms/step; FP32+learned vs plain FP64, same GPU",
        "value": t["particle_steps_per_s"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "dtype_detail": "f32 particle state and gather/push/deposit arithmetic, f64 current "
                        "accumulation, fields, CG and diagnostics; learned aid ("
                        + args.learned_form + ")",
        "data": "synthetic (seeded Maxwell-Juettner pair plasma, loaded on the device)",
        "config": {"workload": HEADLINE["label"], "particles": n_part, "cells": HEADLINE["nx"] * HEADLINE["ny"],
                   "tile": list(HEADLINE_TILE), "tile_split": HEADLINE_SPLIT, "sort_every": HEADLINE_SORT,
                   "cg_rtol": 1e-8},
        "field_solve_ms_per_step": t["field_solve_ms"],
        "cg_iters_last_step": t["cg_iters"],
        "roofline": {"bound": "hbm", "kernel": "k_particles (fused gather+Boris+move+deposit)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "bytes per launch", "traffic_source": traffic_src,
                     "bytes_per_particle_step": BYTES_PER_PARTICLE["fp32"],
                     "algorithmic_bytes_per_launch": alg, "avg_launch_ms": t["push_ms"],
                     "launches_timed": t["push_launches"],
                     "ceilings": ceilings(rec, n_part, t["push_ms"])},
        "headline": h,
        "cpu_baseline": cpu,
    }
    line.update(legs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
