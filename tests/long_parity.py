"""Long runs of the workload files against the oracle (test infrastructure;
not collected by pytest: a 500-step 128^3 oracle run takes a quarter of an hour).

    python -m tests.long_parity run c1_revolving_plate_128 --out oracle.jsonl [--steps N]
    python -m tests.long_parity compare ref.jsonl run.jsonl [run2.jsonl ...]

``run`` writes the oracle's run of the workload in the format of
paper_2002_08642_amd.run (same inputs, the oracle's own adaptive dt: FP64
everywhere, numpy FFTs of oracle.ns, FD-Jacobian Newton of oracle.structure
for the wing).  ``compare`` prints, for every other log against the first, the
largest relative differences of dt, F (relative to max |F| over the steps so
far), E and umax over windows of steps, and of the wing deflection.
"""

import argparse
import json
import sys
import time

import numpy as np

import synth
from oracle import kinematics, ns as ons, structure as st
from oracle.coupling import CoupledOracle


def oracle_run(cfg, steps, emit, progress=None):
    kind = cfg["kind"]
    case = cfg["case"]
    if kind == "taylor_green":
        o = ons.OracleNS(case["n"], case["L"], case["nu"], case["eta"], case["tw"], case["h"], case["profile"])
        o.set_velocity(synth.taylor_green_3d(case["n"], case["L"]))
        x, v, tri = case["wing"]
        o.set_wing(x, v, tri)
        t = 0.0
        for k in range(steps):
            d = o.step(dt=cfg["dt"])
            emit(_line(k, t, d))
            t += d["dt"]
            if progress:
                progress(k)
        return
    rule = cfg["dt"]
    if kind == "revolving_plate":
        o = ons.OracleNS(case["n"], case["L"], case["nu"], case["eta"], case["tw"], case["h"], case["profile"])
        o.set_velocity(np.zeros((3,) + tuple(case["n"])[::-1]))
        t = 0.0
        for k in range(steps):
            x, v = kinematics.plate_pose(case["span_coord"], case["chord_coord"], t, case["alpha"], case["omega"],
                                         case["t_ramp"], case["axis_point"])
            o.set_wing(x, v, case["tri"])
            d = o.step(cfl=rule["cfl"], c_eta=rule["c_eta"], dt_max=rule["dt_max"])
            emit(_line(k, t, d))
            t += d["dt"]
            if progress:
                progress(k)
        return
    if kind == "flexible_wing":
        w = cfg["wing_net"]
        ijk, owner = synth.vein_bending(w)
        kb = np.array([st.bending_stiffness(w["vein_EI"][v], w["vein_length"], len(w["veins"][v]) - 2)
                       for v in owner])
        kin = dict(alpha=case["alpha"], omega=case["omega"], t_ramp=case["t_ramp"], axis_point=case["axis_point"])
        o = CoupledOracle(case["n"], case["L"], case["nu"], case["eta"], case["tw"], case["h"], case["profile"], w,
                          ijk, kb, np.zeros(len(ijk), np.int32), kin, tol=1e-10, order=cfg.get("order", "lagged"))
        o.fluid.set_velocity(np.zeros((3,) + tuple(case["n"])[::-1]))
        for k in range(steps):
            t0 = o.t
            o.step(cfl=rule["cfl"], c_eta=rule["c_eta"], dt_max=rule["dt_max"])
            xr, _ = o._root_pose(o.t, None)
            emit(_line(k, t0, o.last, {"deflection": float(np.max(np.linalg.norm(o.q[0] - xr, axis=1)))}))
            if progress:
                progress(k)
        return
    raise ValueError("no oracle run for workload kind %r" % kind)


def _line(k, t, d, extra=None):
    r = {"step": k, "t": t, "dt": float(d["dt"]), "E": float(d["E"]), "umax": float(d["umax"]),
         "F": [float(f) for f in d["F"]]}
    if extra:
        r.update(extra)
    return r


def load(path):
    with open(path) as f:
        lines = [json.loads(l) for l in f if l.strip()]
    return lines[0], lines[1:]


def compare(ref_path, paths, windows=(20, 100, 200, 300, 500)):
    h0, ref = load(ref_path)
    print("reference: %s (%s, %d steps)" % (ref_path, h0.get("prec", "oracle"), len(ref)))
    F0 = np.array([r["F"] for r in ref])
    out = {}
    for p in paths:
        h, run = load(p)
        n = min(len(ref), len(run))
        F = np.array([r["F"] for r in run[:n]])
        rows = []
        for wdw in sorted(set([w for w in windows if w <= n] + [n])):
            sl = slice(0, wdw)
            scale = np.max(np.abs(F0[sl]))
            row = dict(steps=wdw,
                       dt=max(abs(a["dt"] - b["dt"]) / b["dt"] for a, b in zip(run[sl], ref[sl])),
                       F=float(np.max(np.abs(F[sl] - F0[sl])) / scale) if scale > 0 else 0.0,
                       E=max(abs(a["E"] - b["E"]) / max(abs(b["E"]), 1e-300) for a, b in zip(run[sl], ref[sl])),
                       umax=max(abs(a["umax"] - b["umax"]) / max(abs(b["umax"]), 1e-300)
                                for a, b in zip(run[sl], ref[sl])),
                       t_end=run[wdw - 1]["t"] + run[wdw - 1]["dt"])
            if "deflection" in ref[0] and "deflection" in run[0]:
                dref = np.array([r["deflection"] for r in ref[sl]])
                drun = np.array([r["deflection"] for r in run[sl]])
                row["deflection"] = float(np.max(np.abs(drun - dref)) / max(np.max(np.abs(dref)), 1e-300))
            rows.append(row)
        out[p] = rows
        print("%s (%s):" % (p, h.get("prec", "oracle")))
        for r in rows:
            print("  steps %4d (t = %.4f): dt %.2e  F %.2e  E %.2e  umax %.2e%s"
                  % (r["steps"], r["t_end"], r["dt"], r["F"], r["E"], r["umax"],
                     "  deflection %.2e" % r["deflection"] if "deflection" in r else ""))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("config")
    r.add_argument("--steps", type=int, default=None)
    r.add_argument("--out", required=True)
    c = sub.add_parser("compare")
    c.add_argument("ref")
    c.add_argument("runs", nargs="+")
    a = ap.parse_args(argv)
    if a.cmd == "compare":
        compare(a.ref, a.runs)
        return 0
    cfg = synth.load_config(a.config)
    steps = int(a.steps if a.steps is not None else cfg["steps"])
    t0 = time.time()
    with open(a.out, "w") as f:
        f.write(json.dumps({"workload": cfg["name"], "kind": cfg["kind"], "prec": "oracle-fp64", "steps": steps,
                            "n": cfg.get("n")}) + "\n")

        def emit(d):
            f.write(json.dumps(d) + "\n")
            f.flush()

        def progress(k):
            if (k + 1) % 10 == 0 or k + 1 == steps:
                print("oracle %s: step %d/%d, %.1f s" % (cfg["name"], k + 1, steps, time.time() - t0), flush=True)

        oracle_run(cfg, steps, emit, progress)
    return 0


if __name__ == "__main__":
    sys.exit(main())
