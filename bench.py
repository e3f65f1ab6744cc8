#!/usr/bin/env python3
"""Throughput of the penalized pseudo-spectral Navier-Stokes step on one MI355X.

Workload (512^3 by default): periodic box of side 12 (four plate spans), a
random divergence-free velocity field with a k^(-5/3) spectrum and unit
energy, and the rigid revolving plate (span 3, chord 1, 45 deg pitch,
41 x 13 vertices = 960 triangles) turning at full speed Omega = 2 pi; nu =
pi/300 (Re = 1800), eta = 2.5e-3 (128/N)^2, cosine mask with t_w = 2 dx,
h = dx; adaptive dt (CFL 0.1, C_eta 2/3, dt_max 1e-2).  One step = host pose
of the plate at t^n, mesh upload, mask rebuild, the five transform passes,
reductions and device-side dt, and the read-back of dt / forces that the next
pose needs.

Prints one JSON line: Mpts/s (FP32 bulk with FP64 reductions) with the FP64
run beside it, the roofline of the dominant kernel (HIP events on the library
stream, algorithmic bytes of that pass), and the FP64 CPU oracle timed on a
bounded sample of the same workload.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def workload(n):
    import synth
    cfg = synth.revolving_plate(n=n, t_ramp=0.0)
    return cfg


def algorithmic_bytes(n, wsize, cells):
    """Bytes each pass must move (unpadded layouts), per launch."""
    K = (n - 1) // 3
    kx1, nb = K + 1, 2 * K + 1
    c = 2 * wsize  # complex value
    compact = nb * nb * kx1 * c
    zslab = n * nb * kx1 * c       # [z][iy][ix]
    yslab = n * n * kx1 * c        # [z][y][ix]
    # After the first step the z inverse of the next step (5 z-slab fields written)
    # runs inside the z-forward/update pass, from the new velocity in registers;
    # "z_inverse_curl" is the stand-alone pass of a first step.
    return {
        "z_inverse_curl": 3 * compact + 5 * zslab,
        "y_inverse": 5 * zslab + 6 * yslab,
        "x_fused": 9 * yslab + 4 * cells * wsize,
        "y_forward": 3 * yslab + 3 * zslab,
        "z_forward_update": 3 * zslab + 12 * compact + 5 * zslab,
    }


def step_model_bytes(n, wsize):
    """Whole-step pass model (one HBM round trip per axis pass, 5 fields after z)."""
    K = (n - 1) // 3
    kx1, nb = K + 1, 2 * K + 1
    c = 2 * wsize
    compact = nb * nb * kx1 * c
    zslab = n * nb * kx1 * c
    yslab = n * n * kx1 * c
    return (3 * compact + 5 * zslab) + (5 * zslab + 6 * yslab) + 9 * yslab + (3 * yslab + 3 * zslab) \
        + (3 * zslab + 12 * compact)


def design_step_bytes(n, wsize):
    """Bytes a step of this design moves: the pass model without P1's reads of the
    three compact components (the fused update pass has them in registers)."""
    K = (n - 1) // 3
    kx1, nb = K + 1, 2 * K + 1
    return step_model_bytes(n, wsize) - 3 * nb * nb * kx1 * 2 * wsize


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "fft_lds.h", "wave512.h", "device_util.h", "kernels.h", "launch.h", "engine.hip"):
        with open(os.path.join(ROOT, "paper_2002_08642_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def sponge_layers(n):
    """Sponge of the optional leg: cosine layers n/8 deep at the two x faces and at the top z face."""
    w = max(2, n // 8)
    i = np.arange(n)
    d = np.minimum(i, n - i) / float(w)
    gx = np.where(d < 1.0, 0.5 * (1.0 + np.cos(np.pi * d)), 0.0)
    dz = (n - 1 - i) / float(w)
    gz = np.where(dz < 1.0, 0.5 * (1.0 + np.cos(np.pi * dz)), 0.0)
    return gx, gz


SPONGE_C = 1e-2  # C_sp of the sponge leg (dt / C_sp ~ 0.01 on this workload)


def run_gpu(n, prec, steps, warmup, timing, sponge=False, uh0=None):
    from paper_2002_08642_amd import fsi
    import synth
    cfg = workload(n)
    s = fsi.Solver(cfg["n"], cfg["L"], cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"], prec)
    s.set_spectrum(synth.random_solenoidal_compact(cfg["n"], cfg["L"], seed=0) if uh0 is None else uh0)
    if sponge:
        gx, gz = sponge_layers(n)
        s.set_sponge(SPONGE_C, gx=gx, gz=gz)
    t = 0.0

    def one_step(t):
        x, v, _ = fsi.plate_pose(cfg["span_coord"], cfg["chord_coord"], t, cfg["alpha"], cfg["omega"],
                                 0.0, cfg["axis_point"])
        s.set_wing(x, v, cfg["tri"])
        s.step_adaptive(cfg["cfl"], cfg["c_eta"], cfg["dt_max"])
        info = s.info()
        return t + info["dt"], info

    for _ in range(warmup):
        t, info = one_step(t)
    per_pass, dominant = {}, None
    if timing:
        # every pass timed on a few steps before the timed region; inside it only
        # the pass with the largest time (each recorded event orders its stream)
        s.synchronize()
        s.set_timing(True)
        for _ in range(SAMPLE_STEPS):
            t, info = one_step(t)
        passes, nrec = s.pass_times()
        per_pass = {k: v / max(nrec, 1) for k, v in passes.items()}
        dominant = max(per_pass, key=per_pass.get)
        s.set_timing(True, passes=[dominant])
    s.synchronize()
    sync_torch()
    t0 = time.perf_counter()
    for _ in range(steps):
        t, info = one_step(t)
    s.synchronize()
    sync_torch()
    el = time.perf_counter() - t0
    if timing:
        passes, nrec = s.pass_times()
        per_pass[dominant] = passes[dominant] / max(nrec, 1)
        s.set_timing(False)
    s.close()
    return el / steps, per_pass, info, dominant


SAMPLE_STEPS = 5  # steps with every pass timed, before the timed region


def large_grid_leg(n, steps, warmup):
    """The same workload at n^3 (800^3: 2^5 5^2, run-time mixed-radix plans)
    in FP32 and FP64: time per step, the pass-model roofline fraction of the
    step and the algorithmic-byte rate of every pass."""
    from paper_2002_08642_amd import fsi
    import synth
    cfg = workload(n)
    uh0 = synth.random_solenoidal_compact(cfg["n"], cfg["L"], seed=0)
    out = {"grid": [n, n, n], "steps": steps, "warmup": warmup}
    for name, prec, wsize in (("fp32", fsi.PREC_FP32, 4), ("fp64", fsi.PREC_FP64, 8)):
        ms, passes, _, _ = run_gpu(n, prec, steps, warmup, True, uh0=uh0)
        algo = algorithmic_bytes(n, wsize, 0)
        out[name] = {
            "value": round(n ** 3 / ms / 1e6, 1), "unit": "Mpts/s", "ms_per_step": round(ms * 1e3, 4),
            "step_roofline_frac": round(step_model_bytes(n, wsize) / ms / 1e9 / HBM_PEAK_GBS, 4),
            "pass_ms": {k: round(v, 4) for k, v in passes.items()},
            "pass_frac": {k: round(algo[k] / (v * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                          for k, v in passes.items() if k in algo and v > 0.01},
        }
    return out


def run_adjoint(n, prec, K):
    """Cost of the checkpointed adjoint relative to the forward step.

    One segment of K fixed-dt steps (dt = C_eta eta, the cap that binds on
    this workload) of the revolving plate in the k^-5/3 field: the forward
    steps (pose, mesh upload, mask, step, force read-back; checkpoint saved)
    against the reverse of the same segment (reload, K recomputed steps with
    tape saves, K adjoint steps with the host pose derivative).  Both legs are
    timed after one untimed rollout that allocates the tape and the adjoint
    buffers."""
    from paper_2002_08642_amd import fsi
    from paper_2002_08642_amd.rollout import PlateRollout
    import synth
    cfg = workload(n)
    s = fsi.Solver(cfg["n"], cfg["L"], cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"], prec)
    dt = cfg["c_eta"] * cfg["eta"]
    ro = PlateRollout(s, cfg, [dt] * K, K=K, uh0=synth.random_solenoidal_compact(cfg["n"], cfg["L"], seed=0))
    a = cfg["alpha"]
    ro.forward(a)
    ro.backward(a)
    ro._reset()
    s.synchronize()
    sync_torch()
    t0 = time.perf_counter()
    for k in range(K):
        if k == 0:
            s.save(0)
        ro._step(k, a)
    s.synchronize()
    tf = time.perf_counter() - t0
    s.adjoint_set(None, None)
    t0 = time.perf_counter()
    g = ro.reverse_segment(0, a)
    s.synchronize()
    tb = time.perf_counter() - t0
    return {"grid": [n, n, n], "segment_steps": K, "dt": dt,
            "forward_ms_per_step": round(tf / K * 1e3, 4),
            "backward_ms_per_step": round(tb / K * 1e3, 4),
            "ratio": round(tb / tf, 3),
            "dJ_dalpha_segment": g,
            "note": "backward = reload + K recomputed steps with tape saves + K adjoint steps"}


_torch = None


def sync_torch():
    global _torch
    if os.environ.get("FSI_BENCH_NO_TORCH"):
        return
    if _torch is None:
        try:
            import torch
            _torch = torch if torch.cuda.is_available() else False
        except Exception:
            _torch = False
    if _torch:
        _torch.cuda.synchronize()


def cpu_baseline(n_sample):
    import numpy as np
    import synth
    from oracle import ns, kinematics
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 0) for p in threadpool_info()] or [os.cpu_count()])
    except Exception:
        threads = os.cpu_count()
    cfg = workload(n_sample)
    o = ns.OracleNS(cfg["n"], cfg["L"], cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"])
    o.set_velocity(synth.random_solenoidal(cfg["n"], cfg["L"], seed=0))
    nsteps = 3
    t = 0.0
    t0 = time.perf_counter()
    for _ in range(nsteps):
        x, v = kinematics.plate_pose(cfg["span_coord"], cfg["chord_coord"], t, cfg["alpha"], cfg["omega"], 0.0,
                                     cfg["axis_point"])
        o.set_wing(x, v, cfg["tri"])
        t += o.step(cfl=cfg["cfl"], c_eta=cfg["c_eta"], dt_max=cfg["dt_max"])["dt"]
    el = (time.perf_counter() - t0) / nsteps
    return {"value": n_sample ** 3 / el / 1e6, "unit": "Mpts/s", "cores": int(threads), "kind": "oracle",
            "sample": "%d full oracle steps (mask, naive matrix DFTs, update) of the same workload recipe at "
                      "%d^3, %.1f s each; the 512^3 oracle step needs ~40 GB and minutes" % (nsteps, n_sample, el)}


def load_traffic(n, dominant, wsize):
    path = os.path.join(ROOT, "profiles", "pmc_%d_fp32.json" % n)
    if wsize != 4 or not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            d = json.load(fh)
        if d.get("source_hash") != kernel_source_hash():
            return None
        k = d["kernels"].get(dominant)
        if not k:
            return None
        return k["bytes_per_dispatch"]
    except Exception:
        return None


def calibrate_copy():
    """A plain 1 GiB device-to-device copy (the runtime's copy kernel), for scaling
    the HBM byte counters read under rocprofv3."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    nbytes = 1 << 30
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(a), ctypes.c_size_t(nbytes)) == 0
    assert hip.hipMalloc(ctypes.byref(b), ctypes.c_size_t(nbytes)) == 0
    assert hip.hipMemcpy(b, a, ctypes.c_size_t(nbytes), 3) == 0  # hipMemcpyDeviceToDevice
    assert hip.hipDeviceSynchronize() == 0
    hip.hipFree(a)
    hip.hipFree(b)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--fp64-steps", type=int, default=10)
    ap.add_argument("--cpu-sample", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--adjoint-k", type=int, default=10,
                    help="steps in the timed adjoint segment (0 skips the adjoint/forward leg)")
    ap.add_argument("--sponge-steps", type=int, default=10,
                    help="timed steps of the leg with the vorticity sponge on (0 skips it)")
    ap.add_argument("--large-n", type=int, default=800,
                    help="grid of the large-grid FP32/FP64 leg (800: the largest workload grid)")
    ap.add_argument("--large-steps", type=int, default=10,
                    help="timed steps of the large-grid leg (0 skips it)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 1 GiB device copy first (counter calibration under rocprofv3)")
    ap.add_argument("--no-torch", action="store_true",
                    help="synchronize through the library only (counter collection runs)")
    args = ap.parse_args()
    if args.no_torch:
        os.environ["FSI_BENCH_NO_TORCH"] = "1"
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus must be 1)",
              file=sys.stderr)
        sys.exit(2)
    from paper_2002_08642_amd import fsi
    fsi.load_library()
    if args.calibrate_copy:
        calibrate_copy()

    n = args.n
    ms32, pass32, info32, dominant = run_gpu(n, fsi.PREC_FP32, args.steps, args.warmup, True)
    ms64, pass64 = None, {}
    if args.fp64_steps > 0:
        ms64, pass64, _, _ = run_gpu(n, fsi.PREC_FP64, args.fp64_steps, 2, True)

    adj = run_adjoint(n, fsi.PREC_FP32, args.adjoint_k) if args.adjoint_k > 0 else None
    spg = None
    if args.sponge_steps > 0:
        mss, passs, _, _ = run_gpu(n, fsi.PREC_FP32, args.sponge_steps, 2, True, sponge=True)
        spg = {"value": round(n ** 3 / mss / 1e6, 1), "unit": "Mpts/s", "ms_per_step": round(mss * 1e3, 4),
               "steps": args.sponge_steps, "c_sp": SPONGE_C,
               "layers": "cosine layers n/8 deep at both x faces and the top z face",
               "pass_ms": {k: round(v, 4) for k, v in passs.items()}}

    large = large_grid_leg(args.large_n, args.large_steps, 2) if args.large_steps > 0 else None

    cfg = workload(n)
    # sub-box cells of the mask (chi + 3 u_s read by the fused x pass)
    dx = cfg["L"][0] / n
    cells = 0
    try:
        x, v, _ = fsi.plate_pose(cfg["span_coord"], cfg["chord_coord"], 0.0, cfg["alpha"], cfg["omega"], 0.0,
                                 cfg["axis_point"])
        r = cfg["tw"] + cfg["h"]
        span = (x.max(axis=0) + r) - (x.min(axis=0) - r)
        cells = int(math.prod(int(math.ceil(sv / dx)) + 2 for sv in span))
    except Exception:
        pass
    algo = algorithmic_bytes(n, 4, cells)
    t_dom = pass32[dominant] * 1e-3
    achieved = algo.get(dominant, 0) / t_dom / 1e9 if dominant in algo else None
    traffic = load_traffic(n, dominant, 4)
    model = step_model_bytes(n, 4)
    value = n ** 3 / (ms32) / 1e6
    out = {
        "metric": "Mpts/s per full NS step at %d^3 (FP32 bulk, FP64 reductions)" % n,
        "value": round(value, 1),
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32 * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "revolving rigid plate in k^-5/3 turbulence, %d^3 periodic box" % n,
                   "grid": [n, n, n], "box": cfg["L"][0], "triangles": int(len(cfg["tri"])),
                   "nu": cfg["nu"], "eta": cfg["eta"], "dt": "adaptive (CFL 0.1, C_eta 2/3)",
                   "parallelism": "single GPU"},
        "roofline": {
            "bound": "hbm",
            "kernel": dominant,
            "achieved": None if achieved is None else round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": None if achieved is None else round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes": algo.get(dominant),
            "launch_ms": round(pass32[dominant], 4),
        },
        "step_roofline": {
            # model_bytes: one HBM round trip per axis pass (frac: the equivalent
            # rate); design_bytes: what this implementation moves per step
            "model_bytes": model,
            "frac": round(model / ms32 / 1e9 / HBM_PEAK_GBS, 4),
            "design_bytes": design_step_bytes(n, 4),
            "design_frac": round(design_step_bytes(n, 4) / ms32 / 1e9 / HBM_PEAK_GBS, 4),
            "pass_ms": {k: round(v, 4) for k, v in pass32.items()},
            "pass_ms_note": "HIP-event times per pass on %d steps before the timed region, except the "
                            "dominant pass, timed in the timed region" % SAMPLE_STEPS,
        },
        "fp64": None if ms64 is None else {
            "value": round(n ** 3 / ms64 / 1e6, 1), "unit": "Mpts/s", "ms_per_step": round(ms64 * 1e3, 4),
            "steps": args.fp64_steps,
            "step_roofline_frac": round(step_model_bytes(n, 8) / ms64 / 1e9 / HBM_PEAK_GBS, 4),
            "pass_ms": {k: round(v, 4) for k, v in pass64.items()},
        },
        "adjoint": adj,
        "sponge": spg,
        "large_grid": large,
        "last_step": {"dt": info32["dt"], "umax": info32["umax"], "E": info32["E"],
                      "F": [float(f) for f in info32["F"]]},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
