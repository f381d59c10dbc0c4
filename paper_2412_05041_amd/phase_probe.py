"""Per-phase timing of the track finder (diagnostic).

Loads the phase-timing build of the library (build.py --phase-timing ->
libvelo_phase.so, the same kernels with wall-clock counters read after a
barrier at the end of each phase of a plane step), runs the pipeline on a
synthetic batch and prints, for each finder pass, the time per event of each
phase (microseconds of one workgroup, summed over the 26 plane steps) and the
downstream-completion step counts, as markdown.

    python -m paper_2412_05041_amd.phase_probe [--workload nominal] [--launch 256,0] [--reps 5]

The counters tick at 100 MHz.  The barriers they add make the whole run
slower than the product build; the split between phases is what they show.
"""
import argparse
import ctypes as C
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

PASSES = ("first LDS tile", "second LDS tile (512 threads)", "global memory")
PHASES = ("plane load", "forwarding (T1)", "seed enumeration (T2)", "seed filter + claiming (T2)",
          "track creation + downstream completion (T3)")
TICK_US = 0.01  # 100 MHz


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", default="nominal")
    ap.add_argument("--launch", default="256,0")
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    from paper_2412_05041_amd import build, gen, velo
    if not os.path.exists(build.PHASE_LIB):
        build.build(phase_timing=True)
    velo.LIB_PATH = build.PHASE_LIB
    import torch
    lib = velo.lib()
    lib.velo_probe_phase.argtypes = [C.c_void_p, C.c_int]
    w = gen.WORKLOADS[a.workload]
    b = gen.generate(w)
    cuts = json.load(open(os.path.join(HERE, "configs", "cuts_ms.json" if w.ms_sigma > 0 else "cuts_default.json")))
    v = velo.Velo(b.plane_z, cuts)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    th, tl = (int(x) for x in a.launch.split(","))
    v.set_launch(th, tl)
    off, ids = velo.to_device(b)
    bufs = v.pipeline_buffers(b.n_events, b.n_pix)
    v.pipeline(off, ids, bufs)
    torch.cuda.synchronize()
    buf = (C.c_ulonglong * 36)()
    if lib.velo_probe_phase(buf, 1) != 0:
        raise RuntimeError("velo_probe_phase failed")
    for _ in range(a.reps):
        v.pipeline(off, ids, bufs)
    torch.cuda.synchronize()
    if lib.velo_probe_phase(buf, 1) != 0:
        raise RuntimeError("velo_probe_phase failed")
    st = v.read_status(bufs["status"])
    assert st[0] == 0, st[:8]
    g = [[buf[p * 12 + i] for i in range(12)] for p in range(3)]
    print(f"Workload {a.workload}: {b.n_events} events, {int(st[1]) / b.n_events:.0f} clusters/event; "
          f"launch {th} threads x tile {tl}; {a.reps} pipeline runs; phase-timing build.\n")
    print("| pass | events | us/event (whole) | plane load: ring write | " + " | ".join(PHASES) +
          " | T3 steps/event on ring, other planes | us/event in T3 steps on other planes |")
    print("|---|---|---|---|" + "---|" * len(PHASES) + "---|---|")
    for p in range(3):
        ev = g[p][8]
        if not ev:
            continue
        per = [g[p][i] * TICK_US / ev for i in range(5)]
        ring = g[p][10] * TICK_US / ev
        per[0] += ring  # the plane load: ring write, then issuing the prefetch
        whole = g[p][9] * TICK_US / ev
        tot = sum(per)
        cells = " | ".join(f"{x:.1f} ({100 * x / tot:.0f} %)" for x in per)
        print(f"| {PASSES[p]} | {ev // a.reps} | {whole:.1f} | {ring:.1f} | {cells} | "
              f"{g[p][5] / ev:.1f}, {g[p][6] / ev:.1f} | {g[p][7] * TICK_US / ev:.1f} |")


if __name__ == "__main__":
    main()
