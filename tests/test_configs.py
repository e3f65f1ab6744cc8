"""The workload files (configs/*.json) agree with the inputs the tests build
(synth) and with each other: grid, box, viscosity from Re = 1800, eta from
constant K_eta, the adaptive-dt rule, the wing and plate parameters."""

import json
import math
import os

import numpy as np
import pytest

import synth

NAMES = ["c0_taylor_green_32", "c1_revolving_plate_128", "c2_flexible_wing_256", "c3_throughput_512_800",
         "c4_hinge_plate_128"]


@pytest.mark.parametrize("name", NAMES)
def test_files_load_and_name_themselves(name):
    c = synth.load_config(name)
    assert c["name"] == name
    with open(os.path.join(synth.CONFIG_DIR, name + ".json")) as f:
        assert json.load(f)["kind"] == c["kind"]


def test_revolving_plate_parameters():
    for name, n in (("c1_revolving_plate_128", 128), ("c2_flexible_wing_256", 256), ("c4_hinge_plate_128", 128)):
        c = synth.load_config(name)
        case = c["case"]
        assert case["n"] == (n, n, n) and case["L"] == (12.0,) * 3
        # Re = Omega R c / nu = 1800 with Omega = 2 pi, R = 3, c = 1
        assert case["omega"] * 3.0 * 1.0 / case["nu"] == pytest.approx(1800.0, rel=1e-14)
        assert case["eta"] == pytest.approx(2.5e-3 * (128.0 / n) ** 2, rel=1e-15)
        # K_eta = sqrt(nu eta) / dx is the same at every grid
        assert math.sqrt(case["nu"] * case["eta"]) / (12.0 / n) == pytest.approx(0.0546, abs=5e-4)
        if c["dt"]["rule"] == "adaptive":
            for k in ("cfl", "c_eta", "dt_max"):
                assert c["dt"][k] == pytest.approx(case[k], rel=1e-15)
    c1 = synth.load_config("c1_revolving_plate_128")
    # the ramp sweeps 0.2 revolutions: the integral of (1 - cos(pi t / T)) / 2 over T is T / 2
    assert c1["case"]["omega"] * c1["t_ramp"] / 2 / (2 * math.pi) == pytest.approx(0.2, rel=1e-14)
    assert len(c1["case"]["tri"]) == 2 * 40 * 12


def test_flexible_wing_parameters():
    c = synth.load_config("c2_flexible_wing_256")
    w, ref = c["wing_net"], synth.flexible_wing(density=1.0)
    for k in ("ext_k", "vein_EI", "clamped", "tri", "ext_ij"):
        assert np.array_equal(np.asarray(w[k]), np.asarray(ref[k])), k
    assert len(w["veins"]) == 8 and all(len(v) == 25 for v in w["veins"])
    assert len(w["tri"]) == 2 * 30 * 15
    scale = synth.structure_units()
    assert np.all(w["vein_EI"] / scale >= 1e-3) and np.all(w["vein_EI"] / scale <= 1e-1)


def test_hinge_and_taylor_green_parameters():
    c = synth.load_config("c4_hinge_plate_128")
    p, ref = c["plate_net"], synth.hinge_plate(density=1.0)
    for k in ("bend_kb", "bend_group", "ext_k"):
        assert np.array_equal(np.asarray(p[k]), np.asarray(ref[k])), k
    assert c["case"]["t_ramp"] == 0.2 and c["steps"] == 50 and c["checkpoint_every"] == 10
    c0 = synth.load_config("c0_taylor_green_32")
    case = c0["case"]
    assert case["n"] == (32,) * 3 and case["nu"] == c0["nu"] and case["dt"] == c0["dt"] and case["steps"] == 20
