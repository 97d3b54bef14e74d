"""Host-side checks of the HIP library (no GPU needed).

- libsusp.so loads and exports every function that include/susp.h declares,
- parameter validation that runs before any device call (susp_footprint_bytes),
- the footprint grows with the lattice and the precision as the device layout says.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "susp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(susp_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def susp():
    from paper_1904_02929_amd import susp as S
    if not os.path.exists(S.LIB_PATH):
        pytest.skip("libsusp.so is not built")
    return S


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("susp_create", "susp_step", "susp_stress", "susp_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol(susp):
    lib = ctypes.CDLL(susp.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_default_params(susp):
    p = susp.default_params()
    assert p.tau == 1.0 and p.rho0 == 1.0 and p.map_ratio == 0.95
    assert p.n_sub == 8 and p.precision == susp.FP32 and p.shear_kind == 0


@pytest.mark.parametrize("kw, msg", [
    (dict(box=(4, 16, 16)), "at least 8"),
    (dict(box=(16, 16, 16), tau=0.5), "tau"),
    (dict(box=(16, 16, 16), precision=5), "precision"),
    (dict(box=(16, 16, 16), n_sub=0), "n_sub"),
    (dict(box=(16, 16, 16), shear_kind=7), "shear_kind"),
    (dict(box=(512, 512, 256)), "4 GiB"),
    (dict(box=(320, 320, 320), precision=0), "4 GiB"),
])
def test_invalid_parameters_rejected_on_the_host(susp, kw, msg):
    box = kw.pop("box")
    p = susp.make_params(box, **kw)
    with pytest.raises(susp.SuspError) as e:
        susp.footprint_bytes(p)
    assert e.value.code == susp.EINVAL
    assert msg in str(e.value)


def test_sphere_outside_box_rejected(susp):
    import numpy as np
    p = susp.make_params((32, 32, 32), radius=np.array([4.0]), pos=np.array([[40.0, 5.0, 5.0]]))
    with pytest.raises(susp.SuspError):
        susp.footprint_bytes(p)


def test_footprint_scales_with_lattice_and_precision(susp):
    f32 = susp.footprint_bytes(susp.make_params((64, 64, 64)))
    f64 = susp.footprint_bytes(susp.make_params((64, 64, 64), precision=susp.FP64))
    f16 = susp.footprint_bytes(susp.make_params((64, 64, 64), precision=susp.FP16STORE))
    nodes = 64 ** 3
    # two population arrays of 19 planes dominate the difference between precisions
    assert f64 - f32 >= 2 * 19 * nodes * 4
    assert f32 - f16 >= 2 * 19 * nodes * 2
    big = susp.footprint_bytes(susp.make_params((128, 64, 64)))
    assert big > 1.9 * f32
