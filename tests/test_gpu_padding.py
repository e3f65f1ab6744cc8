"""No result depends on the padding columns of the spectral buffers (the x
columns beyond the 2/3 band, up to the 128-byte row pitch): with NaN written
into them before every call (fsi_debug_poison_padding), the steps, forces,
energy, spectrum, nonlinear term, pressure loads and the reverse step are bit
for bit those of a run without it.

Shapes: the 512-point x pass with the paired 512-point y passes; the 512-point
update + z-inverse pass with the sponge; generic lengths in FSI mode (pressure
spectrum and loads).  Both precisions.
"""

import numpy as np
import pytest

from paper_2002_08642_amd import fsi
import synth

pytestmark = pytest.mark.gpu

DX = 0.03
CASES = {
    "x512_y512": dict(n=(512, 512, 16)),
    "z512_sponge": dict(n=(48, 16, 512), sponge=True),
    "generic_pressure": dict(n=(96, 64, 48), pressure=True),
}


def make(case, prec, seed=3):
    n = case["n"]
    L = tuple(DX * m for m in n)
    s = fsi.Solver(n, L, 0.01, 0.05, 2 * DX, DX, 0, prec, pressure=case.get("pressure", False))
    if case.get("sponge"):
        z = np.arange(n[2])
        gz = np.clip(1.0 - np.minimum(z, n[2] - 1 - z) / (0.1 * n[2]), 0.0, 1.0)
        s.set_sponge(0.1, gz=gz)
    u0 = synth.random_solenoidal(n, L, seed=seed)
    c = np.array(L) / 2
    x, tri = synth.flat_rectangle(tuple(c), (1, 0, 0), (0, 0, 1), min(0.3, L[0] / 4), min(0.2, L[2] / 4), 5, 4)
    v = np.tile(np.array([0.2, -0.1, 0.3]), (len(x), 1))
    return s, u0, x, v, tri


def run(case, prec, poison):
    s, u0, x, v, tri = make(case, prec)
    out = []

    def pz():
        if poison:
            s.poison_padding(np.nan)

    s.set_velocity(u0)
    s.set_wing(x, v, tri)
    dts = [0.004, 0.005, 0.0045]
    for k, dt in enumerate(dts):
        pz()
        s.step_record(dt, k)
        i = s.info()
        out += [i["F"], np.array([i["E"], i["umax"], i["dt"]])]
        if case.get("pressure"):
            pz()
            out += list(s.pressure_loads())
    pz()
    out += [s.velocity(), s.spectrum(), s.nonlinear()]
    # reverse the last two steps
    rng = np.random.default_rng(5)
    lam = s.spectrum() * (rng.standard_normal(s.spectrum().shape) + 0.0)
    pz()
    s.adjoint_set(lam, None)
    for k in (2, 1):
        pz()
        out += list(s.step_adjoint(k, dts[k], dts[k - 1], 0, (0.3, -0.2, 0.5)))
    pz()
    out += list(s.adjoint_get())
    return out


@pytest.mark.parametrize("prec", [fsi.PREC_FP64, fsi.PREC_FP32])
@pytest.mark.parametrize("name", sorted(CASES))
def test_nan_in_padding_changes_nothing(name, prec):
    print("padding", name, prec, flush=True)
    ref = run(CASES[name], prec, False)
    got = run(CASES[name], prec, True)
    assert len(ref) == len(got)
    for k, (a, b) in enumerate(zip(ref, got)):
        a, b = np.asarray(a), np.asarray(b)
        assert np.all(np.isfinite(a)), k
        assert np.array_equal(a, b), (k, float(np.nanmax(np.abs(a - b))) if a.size else 0.0)
