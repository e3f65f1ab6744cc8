"""fsi_get_mask_noalloc (the entry point that allocates nothing) against
fsi_get_mask through the C ABI: the same mask kernels with the argmin keys in
the library's fixed per-device scratch, written to caller-owned device grids.

Two calls in a row, the second with a smaller wing (fewer sub-box cells: stale
keys of the first call must not leak), in FP32 and FP64; bit-identical to
fsi_get_mask; a wing whose sub-box exceeds the fixed scratch is rejected with
FSI_EINVAL.
"""

import ctypes

import numpy as np
import pytest

from paper_2002_08642_amd import fsi
import synth

pytestmark = pytest.mark.gpu


class DeviceArray:
    """Device memory of the HIP runtime the library uses (test-side allocation)."""

    def __init__(self, shape, dtype):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.shape, self.dtype = tuple(shape), np.dtype(dtype)
        self.nbytes = int(np.prod(self.shape)) * self.dtype.itemsize
        self.ptr = ctypes.c_void_p()
        assert self.hip.hipMalloc(ctypes.byref(self.ptr), ctypes.c_size_t(self.nbytes)) == 0
        # poison: every element must be overwritten by the call
        host = np.full(self.shape, np.nan, dtype=self.dtype)
        assert self.hip.hipMemcpy(self.ptr, host.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(self.nbytes),
                                  1) == 0

    def get(self):
        host = np.empty(self.shape, dtype=self.dtype)
        assert self.hip.hipDeviceSynchronize() == 0
        assert self.hip.hipMemcpy(host.ctypes.data_as(ctypes.c_void_p), self.ptr, ctypes.c_size_t(self.nbytes),
                                  2) == 0
        return host

    def free(self):
        if self.ptr:
            self.hip.hipFree(self.ptr)
            self.ptr = None


def plate(n, L, span, seed):
    cfg = synth.revolving_plate(n=n[0], box=L[0])
    s, c = synth.plate_span_chord(41, 13, span, 1.0)
    x, v, _ = fsi.plate_pose(s, c, 0.37 + seed * 0.11, cfg["alpha"], cfg["omega"], 0.0, cfg["axis_point"])
    return cfg, x, v, synth.grid_triangles(41, 13)


@pytest.mark.parametrize("prec", [fsi.PREC_FP32, fsi.PREC_FP64])
def test_mask_noalloc_matches_get_mask(prec):
    n, L = (96, 96, 80), (12.0, 12.0, 10.0)
    cfg = synth.revolving_plate(n=96)
    s = fsi.Solver(n, L, cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"], prec)
    dt = np.float32 if prec == fsi.PREC_FP32 else np.float64
    nx, ny, nz = n
    chi_d = DeviceArray((nz, ny, nx), dt)
    us_d = DeviceArray((3, nz, ny, nx), dt)
    try:
        cells = []
        for call, span in enumerate((3.0, 1.4)):  # second call: a smaller wing
            print("noalloc mask prec %d call %d span %g" % (prec, call, span), flush=True)
            _, x, v, tri = plate(n, L, span, call)
            s.set_wing(x, v, tri)
            s.mask_noalloc(chi_d.ptr.value, us_d.ptr.value)
            s.synchronize()
            chi_g, us_g = chi_d.get(), us_d.get()
            chi_r, us_r = s.mask()
            assert np.all(np.isfinite(chi_g)) and np.all(np.isfinite(us_g))
            assert np.array_equal(chi_g.astype(np.float64), chi_r)
            assert np.array_equal(us_g.astype(np.float64), us_r)
            cells.append(int(np.count_nonzero(chi_r)))
            assert cells[-1] > 500
        assert cells[1] < cells[0]
        # no wing: zero everywhere
        s.clear_wing()
        s.mask_noalloc(chi_d.ptr.value, us_d.ptr.value)
        s.synchronize()
        assert not np.any(chi_d.get()) and not np.any(us_d.get())
    finally:
        chi_d.free()
        us_d.free()


def test_mask_noalloc_rejects_a_sub_box_beyond_the_scratch():
    n, L = (128, 128, 128), (12.0, 12.0, 12.0)
    s = fsi.Solver(n, L, 0.01, 2.5e-3, 2 * 12.0 / 128, 12.0 / 128, fsi.PROFILE_COS, fsi.PREC_FP32)
    # a plate across the box diagonal: its enlarged bounding box holds ~1.5e6 grid points
    x, tri = synth.flat_rectangle((6.0, 6.0, 6.0), (1, 0, 0), np.array([0, 1, 1]) / np.sqrt(2), 5.4, 7.0, 9, 7)
    s.set_wing(x, np.zeros_like(x), tri)
    chi_d = DeviceArray((128, 128, 128), np.float32)
    us_d = DeviceArray((3, 128, 128, 128), np.float32)
    try:
        with pytest.raises(fsi.FsiError) as e:
            s.mask_noalloc(chi_d.ptr.value, us_d.ptr.value)
        assert e.value.code == -1
        assert "scratch" in str(e.value)
        chi_r, _ = s.mask()  # the allocating entry point still serves it
        assert np.count_nonzero(chi_r) > 1000
    finally:
        chi_d.free()
        us_d.free()
