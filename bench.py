#!/usr/bin/env python
"""VELO hot-path benchmark on one MI355X.

Workload (the nominal-occupancy configuration): 1000 synthetic events, Poisson(5)
primary vertices x Poisson(40) tracks, 1 mrad scattering per plane, calibrated
noise giving ~3k clusters per event (seed 1002).  One step = the whole path
(clustering + staging, track finding, acceptance, CSR output, fit) over the
batch, inputs resident in HBM, launched as one replayed HIP graph; by default four batches are in flight (one
per hardware queue of the process), each on its own context, buffers and HIP
stream (--streams), so that one batch's clustering and output overlap the tail
of another's track finding.

Prints ONE JSON line: events/s, the dominant kernel's HBM roofline fraction
(algorithmic bytes / its HIP-event-timed duration), efficiency / ghost rate of
the output, and the oracle timed on the host cores over a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode plain|learned] [--seed-filter]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# an illustrative magnet for --extrapolate (kink plane, tracker plane in mm; slope
# change per unit q/p in rad GeV; smallest momentum of the window in GeV)
MAGNET = dict(z_mag=5200.0, z_t=7800.0, kick=1.2, p_min=3.0)
METRIC = "VELO events/s at nominal occupancy (1 GPU), eff/ghost rate; % HBM roofline"


def _oracle_chunk(args):
    """CPU baseline worker: the oracle (cluster + find + FP64 fit) on an event slice.
    Returns (events, the finder's brute-force test counts: pairs, triplets, seed candidates)."""
    import numpy as np  # noqa: F401
    import oracle
    pix_off, pix_id, plane_z, cuts, seed = args
    c = oracle.cluster(pix_off, pix_id)
    t = oracle.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], plane_z, cuts, seed=seed)
    oracle.fit(t["trk_hit_off"], t["trk_hit"], t["trk_planes"], c["clu_x"], c["clu_y"], plane_z, cuts["sigma"])
    return int(pix_off.size - 1) // 26, [int(x) for x in t["stats"][:3]]


# Worker processes of the CPU baseline: the host CPUs this process may run on,
# at most 16 -- the host share that goes with one GPU on a shared GPU machine.
MAX_CPU_WORKERS = 16


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(batch, cuts, passes, min_wall, seed=None):
    """The oracle on the host: event-parallel over the worker processes, and on
    one process over a slice of the batch.  Also returns the method's test
    counts per event (brute-force pairs and triplets, from the oracle)."""
    import multiprocessing as mp

    import oracle
    oracle.build()
    avail = len(os.sched_getaffinity(0))
    cores = max(1, min(MAX_CPU_WORKERS, avail))
    chunks = []
    step = max(1, batch.n_events // (cores * 4))
    for e0 in range(0, batch.n_events, step):
        s = batch.event_slice(e0, min(batch.n_events, e0 + step))
        chunks.append((s.pix_off, s.pix_id, batch.plane_z, cuts, seed))
    ctx = mp.get_context("fork")  # no GPU has been touched yet in this process
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_chunk, chunks[:cores])  # warm the workers
        t0 = time.perf_counter()
        n = done = 0
        tests = None
        while done < passes or time.perf_counter() - t0 < min_wall:
            res = pool.map(_oracle_chunk, chunks)
            n += sum(r[0] for r in res)
            if tests is None:
                tests = [sum(r[1][i] for r in res) for i in range(3)]
            done += 1
        dt = time.perf_counter() - t0
    # one process, the first chunk (warm: the pool already ran the oracle once here)
    one = chunks[0]
    _oracle_chunk(one)
    t1 = time.perf_counter()
    n1 = reps1 = 0
    while reps1 < 1 or time.perf_counter() - t1 < min(min_wall, 1.0):
        n1 += _oracle_chunk(one)[0]
        reps1 += 1
    dt1 = time.perf_counter() - t1
    E = batch.n_events
    base = dict(value=n / dt, unit="events/s", cores=cores, kind="oracle",
                sample=f"all {E} events of the benchmark batch x {done} passes "
                       f"(cluster + find + FP64 fit), event-parallel over {cores} worker processes; "
                       f"{dt:.2f} s wall, ~{dt * cores:.0f} s of CPU work",
                host_cpus_available=avail, host_cpu_count=os.cpu_count(), cpu_model=cpu_model(),
                workers_rule=f"min({MAX_CPU_WORKERS}, CPUs this process may run on)",
                one_thread=dict(value=n1 / dt1, unit="events/s",
                                sample=f"events 0..{int(one[0].size - 1) // 26 - 1} x {reps1} passes on one "
                                       f"process, {dt1:.2f} s"))
    per_event = dict(pair_tests=tests[0] / E, triplet_tests=tests[1] / E, seed_candidates=tests[2] / E)
    return base, per_event


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measured_traffic(kernel, launch, workload):
    """HBM bytes per launch from the committed profiler counter runs, or None
    when they were taken for another kernel, launch or workload, or when the
    kernel's sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if rec["kernel"] != kernel or list(rec["launch"]) != list(launch) or h.hexdigest() != rec["sources_sha256"]:
        return None
    return float(rec["traffic_bytes_per_launch"])


def device_copy_gbs(torch, device, mib=1024, reps=10):
    """Attainable HBM bandwidth: a device-to-device copy of `mib` MiB (read +
    write bytes / time), HIP events on the current stream."""
    src = torch.empty(mib << 20, dtype=torch.uint8, device=device)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * src.numel() * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


def describe(w, clusters_per_event):
    """Plain-words description of a synthetic workload."""
    mult = {"fixed": f"{w.n_tracks} tracks/event",
            "pv_poisson": f"Poisson({w.pv_mean:g}) PVs x Poisson({w.trk_per_pv:g}) tracks",
            "lognormal": f"{w.n_tracks} x lognormal(0, {w.ln_sigma:g}) tracks clipped to {list(w.ln_clip)}",
            "uniform": f"single vertex, U[{w.trk_lo}, {w.trk_hi}] tracks"}[w.tracks]
    return (f"{w.name}: {w.n_events} events, {mult}, {w.ms_sigma * 1e3:g} mrad MS/plane, "
            f"noise p={w.noise_p:g} (~{clusters_per_event:.0f} clusters/event), seed {w.seed}")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", choices=["plain", "learned"], default="plain")
    ap.add_argument("--streams", type=int, default=4,
                    help="batches in flight: each on its own context, buffers and HIP stream")
    ap.add_argument("--seed-filter", action="store_true",
                    help="seed-level learned filter with the committed network (configs/seed_default.npz)")
    ap.add_argument("--path", choices=["fused", "three-call"], default="fused",
                    help="fused: velo_pipeline (one replayed HIP graph); three-call: velo_cluster, "
                         "velo_find_tracks, velo_fit launched eagerly")
    ap.add_argument("--workload", default="nominal")
    ap.add_argument("--cpu-passes", type=int, default=1, help="minimum passes of the CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=1.5, help="minimum wall time of the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--launch", default=None, help="threads,tile of the finder (skips the autotuner)")
    ap.add_argument("--raw", action="store_true",
                    help="start each step from super-pixel raw banks: velo_decode, then the path")
    ap.add_argument("--extrapolate", action="store_true",
                    help="also run velo_extrapolate on each step's tracks (an illustrative single-kink magnet)")
    ap.add_argument("--kalman", type=float, default=None, metavar="MS",
                    help="also run velo_kalman_fit on each step's tracks (slope noise per plane, rad)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB 3 times (a known-size kernel that "
                         "scales HBM byte counters read by a profiler)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(events would shard across GPUs with no exchange).", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    from paper_2412_05041_amd import gen, metrics

    cfg = os.path.join(ROOT, "paper_2412_05041_amd", "configs")
    w = gen.WORKLOADS[args.workload]
    cuts = json.load(open(os.path.join(cfg, "cuts_ms.json" if w.ms_sigma > 0 else "cuts_default.json")))
    batch = gen.generate(w)
    E = batch.n_events
    log(f"generated {E} {w.name} events, {batch.n_pix} pixels")

    seed_net = None
    if args.seed_filter:
        d = np.load(os.path.join(cfg, "seed_default.npz"), allow_pickle=False)
        seed_net = (d["weights"].astype(np.float32), d["norm"].astype(np.float32), float(d["threshold"]))

    cpu = tests_per_event = None
    if not args.no_cpu_baseline:
        cpu, tests_per_event = cpu_baseline(batch, cuts, args.cpu_passes, args.cpu_seconds, seed=seed_net)
        log(f"cpu baseline: {cpu['value']:.0f} events/s on {cpu['cores']} cores "
            f"({cpu['one_thread']['value']:.0f} on one)")

    import torch

    from paper_2412_05041_amd import velo

    if args.mode == "learned":
        from paper_2412_05041_amd import learned
        # the network trained on this generator's candidates where there is one
        master, norm = learned.load_default_weights(learned.NOMINAL_WEIGHTS if w.ms_sigma > 0 else learned.WEIGHTS)
        cuts = dict(cuts, mode=1, logit_band=learned.DEFAULT_BAND)
    def new_context():
        c = velo.Velo(batch.plane_z, cuts, device=0)
        if args.mode == "learned":
            c.mlp_set_weights(master, norm)
        if seed_net is not None:
            c.seed_filter_set(*seed_net)
        c.reserve(E, batch.n_pix, batch.n_pix)
        return c

    v = new_context()
    off, ids = velo.to_device(batch)

    bank = None
    if args.raw:
        bank_off, bank = gen.raw_banks(batch, seed=w.seed)
        d_bank_off = torch.from_numpy(bank_off).to(v.device)
        d_bank = torch.from_numpy(bank.view(np.int32)).to(v.device)
        log(f"raw banks: {bank.size} words for {batch.n_pix} pixels")

    class Lane:
        """One batch in flight: a context (workspace, graph), its buffers, its stream."""

        def __init__(self, ctx):
            self.v = ctx
            self.bufs = ctx.pipeline_buffers(E, batch.n_pix)
            self.stream = torch.cuda.Stream()
            self.kal_out = None
            if args.kalman is not None:
                self.kal_out = torch.empty((max(self.bufs["trk_cap"], 1), 16), dtype=torch.float32,
                                           device=ctx.device)
            self.ext_out = None
            if args.extrapolate:
                self.ext_out = torch.empty((max(self.bufs["trk_cap"], 1), 8), dtype=torch.float32,
                                           device=ctx.device)
            self.dec = None
            if bank is not None:
                self.dec = ctx.decode(d_bank_off, d_bank, batch.n_pix)
                self.dec_ids = self.dec["pix_id"][:batch.n_pix]

        def extrapolate(self):
            b = self.bufs
            self.v.extrapolate(b["par"], MAGNET, max_tracks=b["trk_cap"], d_n_tracks=b["trk_off"][E:],
                               out=self.ext_out)

        def kalman(self):
            b = self.bufs
            self.v.kalman_fit(b["trk_hit_off"], b["trk_hit"], b["trk_planes"], b["clu_x"], b["clu_y"], args.kalman,
                              max_tracks=b["trk_cap"], d_n_tracks=b["trk_off"][E:], out=self.kal_out)

        def step(self):
            o, i = off, ids
            if self.dec is not None:
                self.v.decode(d_bank_off, d_bank, batch.n_pix, out=self.dec)
                o, i = self.dec["pix_off"], self.dec_ids
            (self.v.pipeline if args.path == "fused" else self.v.three_call)(o, i, self.bufs)
            if self.kal_out is not None:
                self.kalman()
            if self.ext_out is not None:
                self.extrapolate()

    lanes = [Lane(v)]
    for _ in range(args.streams - 1):
        lanes.append(Lane(new_context()))
    tune_ms = None
    if args.launch:
        th, tl = (int(x) for x in args.launch.split(","))
        for L in lanes:
            L.v.set_launch(th, tl)
    elif not args.no_autotune:
        # the library's autotuner, timing each launch with all batches in flight
        c = v.cluster(off, ids, with_npix=False)
        torch.cuda.synchronize()
        tune_ms, launch = velo.autotune([L.v for L in lanes], c["clu_off"], c["clu_x"], c["clu_y"], reps=8,
                                        streams=[L.stream for L in lanes])
        del c
        log(f"autotune with {len(lanes)} batches in flight: {launch}")
    torch.cuda.synchronize()
    log(f"launch {v.get_launch()}, {args.streams} batch(es) in flight, warm-up")

    cur = torch.cuda.current_stream()

    def run(n):
        # batch k goes to lane k mod N; a lane's batches run in order on its stream
        for L in lanes:
            L.stream.wait_stream(cur)
        for k in range(n):
            L = lanes[k % len(lanes)]
            with torch.cuda.stream(L.stream):
                L.step()
        for L in lanes:
            cur.wait_stream(L.stream)

    run(max(args.warmup, len(lanes)))
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = args.steps * E / dt
    for L in lanes[1:]:
        assert L.v.read_status(L.bufs["status"])[0] == 0
    bufs = lanes[0].bufs
    dec = lanes[0].dec
    kal_out = lanes[0].kal_out
    kalman = lanes[0].kalman
    ext_out = lanes[0].ext_out
    st = v.read_status(bufs["status"])
    if args.path == "three-call":
        stc = v.read_status(bufs["status_clu"])
        st[0] = max(st[0], stc[0])
        st[1] = stc[1]
    if st[0] != 0:
        print(f"status error: {st[:8]}", file=sys.stderr)
        sys.exit(1)

    # outputs, truth matching
    n_clu = int(st[1])
    T = int(st[2])
    H = int(st[3])
    clu_off = bufs["clu_off"].cpu().numpy()
    m = metrics.eff_ghost(batch, bufs["pix_clu"][:batch.n_pix].cpu().numpy(), clu_off,
                          bufs["trk_off"].cpu().numpy(), bufs["trk_hit_off"][:T + 1].cpu().numpy(),
                          bufs["trk_hit"][:H].cpu().numpy())

    # per-stage durations (HIP events on the launch stream, eager launches)
    v.set_timing(True)
    acc = None
    for _ in range(args.steps):
        v.pipeline(off, ids, bufs)
        t = v.last_timing()
        acc = t if acc is None else {k: acc[k] + t[k] for k in acc}
    v.set_timing(False)
    stages = {k: acc[k] / args.steps for k in acc}
    if dec is not None:  # the decode alone, HIP events on the stream it runs on
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            v.decode(d_bank_off, d_bank, batch.n_pix, out=dec)
        e1.record()
        torch.cuda.synchronize()
        stages["decode"] = e0.elapsed_time(e1) / args.steps
        assert v.read_status(dec["status"])[0] == 0
    kal = None
    if kal_out is not None:  # the Kalman fit alone, HIP events on the stream it runs on
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        kalman()
        e0.record()
        for _ in range(args.steps):
            kalman()
        e1.record()
        torch.cuda.synchronize()
        kms = e0.elapsed_time(e1) / args.steps
        stages["kalman"] = kms
        kbytes = 12 * H + 72 * T  # hit index + x, y per hit; offset, planes, 16-float state per track
        kal = {"ms": kms, "alg_bytes": kbytes, "achieved_GBs": kbytes / (kms * 1e-3) / 1e9,
               "frac": kbytes / (kms * 1e-3) / (HBM_PEAK_GBS * 1e9), "ms_noise": args.kalman}
    ext = None
    if ext_out is not None:  # the extrapolation alone, HIP events on the stream it runs on
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        lanes[0].extrapolate()
        e0.record()
        for _ in range(args.steps):
            lanes[0].extrapolate()
        e1.record()
        torch.cuda.synchronize()
        ems = e0.elapsed_time(e1) / args.steps
        stages["extrapolate"] = ems
        ebytes = 52 * T  # x, y, z, tx, ty in; 8 floats out per track
        ext = {"ms": ems, "alg_bytes": ebytes, "achieved_GBs": ebytes / (ems * 1e-3) / 1e9,
               "frac": ebytes / (ems * 1e-3) / (HBM_PEAK_GBS * 1e9), "magnet": MAGNET}
    # dominant kernel: the largest share of the batch's device time -- its
    # duration, for the finder passes weighted by the fraction of the events
    # they process (the second pass takes a few hundred workgroups, not the GPU)
    ev_rest = (st[8:8 + E] & (velo.EV_SECOND_TILE | velo.EV_LARGE_PATH)) != 0
    share = dict(stages)
    share["find_lds"] = stages["find_lds"] * (1.0 - ev_rest.mean())
    share["find_large"] = stages["find_large"] * ev_rest.mean()
    dom = max(("cluster", "find_lds", "find_large", "accept", "output_fit"), key=lambda k: share[k])
    # algorithmic bytes per launch (minimum traffic the stage must move)
    n_pix = batch.n_pix
    # the finder's two stages split the events: those that fit the configured
    # LDS tile, and those that went on to the larger tile or global memory
    clu_ev = np.diff(clu_off[::26].astype(np.int64))
    trk_off_h = bufs["trk_off"].cpu().numpy().astype(np.int64)
    hit_off_h = bufs["trk_hit_off"][:T + 1].cpu().numpy().astype(np.int64)
    trk_ev = np.diff(trk_off_h)
    hit_ev = hit_off_h[trk_off_h[1:]] - hit_off_h[trk_off_h[:-1]]

    def find_bytes(mask):  # hit coordinates in, track hit lists out
        return int(8 * clu_ev[mask].sum() + 4 * hit_ev[mask].sum() + 8 * trk_ev[mask].sum())

    alg = {
        "cluster": 8 * n_pix + 8 * n_clu + 14 * n_clu,    # ids in, labels out, centroids + staging out
        "find_lds": find_bytes(~ev_rest),
        "find_large": find_bytes(ev_rest),
        "accept": 12 * H + 8 * T,                         # gather candidate hits, write flags
        "output_fit": 12 * H + 40 * T,                    # gather hits, write CSR + 8-float state
    }
    achieved = alg[dom] / (stages[dom] * 1e-3) / 1e9
    copy_gbs = device_copy_gbs(torch, v.device)
    log(f"device copy: {copy_gbs:.0f} GB/s")
    alu = None
    if tests_per_event is not None:
        alu = {
            "definition": "the method's brute-force tests (oracle count): every unused (h0, h2) pair of a "
                          "seeding step, every unused middle hit of a pair that passes the pair cuts; the "
                          "GPU's windowed search evaluates the cut only on a subset of them",
            "pair_tests_per_event": tests_per_event["pair_tests"],
            "triplet_tests_per_event": tests_per_event["triplet_tests"],
            "seed_candidates_per_event": tests_per_event["seed_candidates"],
            "pair_tests_per_s": tests_per_event["pair_tests"] * value,
            "triplet_tests_per_s": tests_per_event["triplet_tests"] * value,
        }
    path_bytes = 8 * n_pix + 8 * n_clu + 4 * H + 36 * T  # fused minimum of the whole path
    th, tl = v.get_launch()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": describe(w, n_clu / E),
            "events": E,
            "pixels_per_event": n_pix / E,
            "clusters_per_event": n_clu / E,
            "tracks_per_event": T / E,
            "mode": args.mode,
            "seed_filter": bool(args.seed_filter),
            "path": args.path,
            "kalman_ms": args.kalman,
            "extrapolate": bool(args.extrapolate),
            "raw_banks": bool(args.raw),
            "launch": {"threads_per_event": th, "tile": tl},
            "autotune_ms_per_batch": tune_ms,
            "autotune": "velo_autotune, every launch timed with all batches in flight",
            "batches_in_flight": args.streams,
        },
        "efficiency": m["efficiency"],
        "ghost_rate": m["ghost_rate"],
        "clone_rate": m["clone_rate"],
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(dom, (th, tl), w.name),
            "alg_bytes": alg[dom],
            "launch_ms": stages[dom],
            "launch_timing": "HIP events around the kernel on its stream, one batch in flight",
            "attainable_copy_GBs": copy_gbs,
            "frac_of_attainable": achieved / copy_gbs,
        },
        "alu": alu,
        "path_hbm_frac": path_bytes / E * value / (HBM_PEAK_GBS * 1e9),
        "stages_ms": stages,
        "events_second_tile_or_large": int(ev_rest.sum()),
        "kalman": kal,
        "extrapolate": ext,
        "cpu_baseline": cpu,
    }
    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib << 20, dtype=torch.uint8, device=v.device)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = src.numel()
        del src, dst
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
