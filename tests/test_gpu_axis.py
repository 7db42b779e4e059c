"""gempic_axis_field on the GPU, through the C ABI: the FP64 on-axis column of
every E and B component equals the same column of gempic_fields bit for bit
(FP64 and FP32 handles, 3-D and 2-D, after a few steps), and the rejections
(component outside 0 .. 5, a buffer shorter than the zeta planes)."""
import ctypes

import numpy as np
import pytest

import workloads
from paper_2509_16793_amd.gempic import GempicError, Sim, lib

pytestmark = pytest.mark.gpu

COMPONENTS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")


@pytest.mark.parametrize("cfg", [workloads.small3d("fp64"), workloads.small3d("fp32"),
                                 workloads.lwfa2d_fp64()], ids=["3d-fp64", "3d-fp32", "2d-fp64"])
def test_axis_equals_the_fields_column(cfg):
    g = Sim(cfg)
    g.step(2)
    F = g.fields(COMPONENTS)
    ny, nx = F["Ex"].shape[1], F["Ex"].shape[2]
    for name in COMPONENTS:
        a = g.axis_field(name)
        assert a.dtype == np.float64 and a.shape == (F[name].shape[0],)
        assert np.array_equal(a, F[name][:, ny // 2, nx // 2].astype(np.float64)), name
    g.close()


def test_rejections():
    g = Sim(workloads.small3d("fp32"))
    with pytest.raises(GempicError):
        g.axis_field("Jx")   # not an E or B component: index 6
    out = np.empty(g.Nz, np.float64)
    ptr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib().gempic_axis_field(g.h, 2, ptr, g.Nz - 1) != 0
    assert lib().gempic_axis_field(g.h, -1, ptr, g.Nz) != 0
    assert lib().gempic_axis_field(g.h, 2, ptr, g.Nz) == 0
    g.close()
