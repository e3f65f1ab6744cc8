"""Run a workload file (configs/<name>.json) through the library and log every
step as one JSON line.

    python -m paper_2002_08642_amd.run c1_revolving_plate_128 --prec fp32 --out c1.jsonl [--steps N]

Kinds:
  taylor_green     the 32^3 Taylor-Green box with its static plate, fixed dt;
  revolving_plate  the rigid plate posed by fsi_plate_pose at the start of
                   every step, dt chosen on the device (fsi_step_adaptive);
  flexible_wing    the mass-spring wing coupled to the flow
                   (FlexibleWingFSI.step_adaptive: the structure step takes
                   the dt the fluid step chose).
The first line is a header (workload, precision, grid, library); each further
line holds step, t (start of the step), dt, E, umax and F of that step (the
diagnostics at t^n), and for the flexible wing the largest deflection from
the rigid pose at t^{n+1} and the Newton iterations of the structure step.
Every computation runs in libfsi; this module only sequences calls.
"""

import argparse
import json
import sys
import time

import numpy as np

from . import fsi
from .coupled import FlexibleWingFSI

PRECS = {"fp32": fsi.PREC_FP32, "fp64": fsi.PREC_FP64}


def _solver(case, prec, pressure=False):
    return fsi.Solver(case["n"], case["L"], case["nu"], case["eta"], case["tw"], case["h"], case["profile"], prec,
                      pressure=pressure)


def _line(k, t, info, extra=None):
    d = {"step": k, "t": t, "dt": info["dt"], "E": info["E"], "umax": info["umax"], "F": [float(f) for f in info["F"]]}
    if extra:
        d.update(extra)
    return d


def run(cfg, prec, steps, emit, progress=None):
    """Run ``steps`` steps of the loaded workload ``cfg`` (synth.load_config) and
    pass one dict per step to ``emit``."""
    kind = cfg["kind"]
    if kind == "taylor_green":
        import synth
        case = cfg["case"]
        s = _solver(case, prec)
        s.set_velocity(synth.taylor_green_3d(case["n"], case["L"]))
        x, v, tri = case["wing"]
        s.set_wing(x, v, tri)
        t = 0.0
        for k in range(steps):
            s.step(cfg["dt"])
            i = s.info()
            emit(_line(k, t, i))
            t += i["dt"]
            if progress:
                progress(k)
        return s
    if kind == "revolving_plate":
        case = cfg["case"]
        rule = cfg["dt"]
        s = _solver(case, prec)
        s.set_velocity(np.zeros((3,) + tuple(case["n"])[::-1]))
        tri = np.asarray(case["tri"])
        t = 0.0
        for k in range(steps):
            x, v, _ = fsi.plate_pose(case["span_coord"], case["chord_coord"], t, case["alpha"], case["omega"],
                                     case["t_ramp"], case["axis_point"])
            s.set_wing(x, v, tri)
            s.step_adaptive(rule["cfl"], rule["c_eta"], rule["dt_max"])
            i = s.info()
            emit(_line(k, t, i))
            t += i["dt"]
            if progress:
                progress(k)
        return s
    if kind == "flexible_wing":
        import synth
        case = cfg["case"]
        rule = cfg["dt"]
        w = cfg["wing_net"]
        ijk, owner = synth.vein_bending(w)
        kb = np.array([fsi.bending_stiffness(w["vein_EI"][v], w["vein_length"], len(w["veins"][v]) - 2)
                       for v in owner])
        kin = dict(alpha=case["alpha"], omega=case["omega"], t_ramp=case["t_ramp"], axis_point=case["axis_point"])
        s = _solver(case, prec, pressure=True)
        s.set_velocity(np.zeros((3,) + tuple(case["n"])[::-1]))
        g = FlexibleWingFSI(s, w, ijk, kb, np.zeros(len(ijk), np.int32), kin, tol=1e-10,
                            order=cfg.get("order", "lagged"))
        for k in range(steps):
            t0 = g.t
            g.step_adaptive(rule["cfl"], rule["c_eta"], rule["dt_max"])
            i = s.info()
            x, _ = g.state()
            xr, _ = g._root_pose(g.t, None)
            emit(_line(k, t0, i, {"deflection": float(np.max(np.linalg.norm(x - xr, axis=1))),
                                  "newton": int(g.iters[-1])}))
            if progress:
                progress(k)
        return g
    raise ValueError("workload kind %r is not a time-stepping run (throughput: bench.py; hinge_plate: "
                     "coupled.HingeRollout)" % kind)


def main(argv=None):
    import synth
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("config", help="configs/<name>.json or its name")
    ap.add_argument("--prec", choices=sorted(PRECS), default="fp32")
    ap.add_argument("--steps", type=int, default=None, help="default: the workload's step count")
    ap.add_argument("--out", required=True, help="JSON-lines log")
    a = ap.parse_args(argv)
    cfg = synth.load_config(a.config)
    steps = int(a.steps if a.steps is not None else cfg["steps"])
    t0 = time.time()
    with open(a.out, "w") as f:
        f.write(json.dumps({"workload": cfg["name"], "kind": cfg["kind"], "prec": a.prec, "steps": steps,
                            "n": cfg.get("n"), "library": fsi.LIB_PATH}) + "\n")

        def emit(d):
            f.write(json.dumps(d) + "\n")

        def progress(k):
            if (k + 1) % 50 == 0 or k + 1 == steps:
                f.flush()
                print("%s %s: step %d/%d, %.1f s" % (cfg["name"], a.prec, k + 1, steps, time.time() - t0), flush=True)

        run(cfg, PRECS[a.prec], steps, emit, progress)
    return 0


if __name__ == "__main__":
    sys.exit(main())
