"""The C-ABI library on the CPU: it loads, exports what include/geoloc.h declares, its
struct layouts match the binding, and argument validation / no-device paths return
status codes without touching a GPU."""
import ctypes
import math
import os
import re
import subprocess
import sys
import textwrap

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "geoloc.h")

from paper_2508_06672_amd import geoloc  # noqa: E402


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|int)\s+(geoloc_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    lib = geoloc.load()
    names = declared_functions()
    assert "geoloc_plan" in names and "geoloc_map" in names and "geoloc_argmax" in names
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", geoloc.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (geoloc_\w+)", out))
    assert set(names) <= exported


def test_struct_layout_matches_header(tmp_path):
    probe = tmp_path / "probe.c"
    probe.write_text(textwrap.dedent(f"""
        #include <stdio.h>
        #include <stddef.h>
        #include "{HEADER}"
        int main(void) {{
          printf("%zu %zu %zu\\n", sizeof(geoloc_desc), sizeof(geoloc_inputs), sizeof(geoloc_plan_info));
          printf("%zu %zu %zu %zu\\n", offsetof(geoloc_desc, lat), offsetof(geoloc_desc, method),
                 offsetof(geoloc_desc, caf_nu_hi_hz), offsetof(geoloc_plan_info, map_ms));
          return 0;
        }}"""))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c11", str(probe), "-o", str(exe)], check=True)
    a, b = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")[:2]
    sizes = [int(x) for x in a.split()]
    offs = [int(x) for x in b.split()]
    assert sizes == [ctypes.sizeof(geoloc.geoloc_desc), ctypes.sizeof(geoloc.geoloc_inputs),
                     ctypes.sizeof(geoloc.geoloc_plan_info)]
    assert offs == [geoloc.geoloc_desc.lat.offset, geoloc.geoloc_desc.method.offset,
                    geoloc.geoloc_desc.caf_nu_hi_hz.offset, geoloc.geoloc_plan_info.map_ms.offset]


def _desc(**kw):
    lat = np.linspace(0.1, 0.2, 5)
    lon = np.linspace(0.3, 0.4, 6)
    d = geoloc.geoloc_desc()
    d.n_rx, d.n_pairs, d.pairs = 2, 0, None
    d.n_samples, d.step_len = 4000, 1000
    d.fs_hz, d.fc_hz = 2e6, 1575.42e6
    d.grid_kind, d.n_rows, d.n_cols = geoloc.GRID_RECT, 5, 6
    d._keep = (lat, lon)
    d.lat = lat.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.lon = lon.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.earth_radius_m, d.alt_m = 6371e3, 0.0
    d.caf_nu_lo_hz = d.caf_nu_hi_hz = math.nan
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("field,value", [
    ("n_rx", 1), ("n_samples", 4001), ("step_len", 0), ("fs_hz", 0.0), ("fc_hz", -1.0), ("n_rows", 0),
    ("grid_kind", 7), ("method", 9), ("delay_mode", 5), ("accum_mode", 3), ("earth_radius_m", float("nan")),
])
def test_invalid_descriptors_return_einval(field, value):
    d = _desc(**{field: value})
    h = ctypes.c_void_p()
    rc = geoloc.load().geoloc_plan(ctypes.byref(d), ctypes.byref(h))
    assert rc == geoloc.EINVAL, (field, rc, geoloc.geoloc_last_error())
    assert h.value is None
    assert geoloc.geoloc_last_error()


def test_invalid_pairs_and_nonfinite_grid():
    bad = np.array([[0, 0]], dtype=np.int32)
    d = _desc(n_pairs=1, pairs=bad.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    h = ctypes.c_void_p()
    assert geoloc.load().geoloc_plan(ctypes.byref(d), ctypes.byref(h)) == geoloc.EINVAL
    lat = np.array([0.1, float("nan"), 0.2, 0.3, 0.4])
    d = _desc()
    d.lat = lat.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert geoloc.load().geoloc_plan(ctypes.byref(d), ctypes.byref(h)) == geoloc.EINVAL
    assert geoloc.load().geoloc_plan(None, ctypes.byref(h)) == geoloc.EINVAL


def test_null_plan_calls_return_estate():
    lib = geoloc.load()
    assert lib.geoloc_destroy(None) == geoloc.ESTATE
    assert lib.geoloc_set_timing(None, 1) == geoloc.ESTATE
    assert lib.geoloc_info(None, None) == geoloc.ESTATE
    for s in (geoloc.OK, geoloc.EINVAL, geoloc.ENAN, geoloc.EDEVICE, 123):
        assert geoloc.geoloc_strerror(s)


def test_no_device_returns_edevice():
    """With every GPU hidden, a valid plan request must fail cleanly with EDEVICE."""
    code = textwrap.dedent(f"""
        import sys; sys.path.insert(0, {ROOT!r})
        sys.path.insert(0, {os.path.join(ROOT, 'tests')!r})
        import ctypes
        from paper_2508_06672_amd import geoloc
        from test_abi_cpu import _desc
        d = _desc(); h = ctypes.c_void_p()
        rc = geoloc.load().geoloc_plan(ctypes.byref(d), ctypes.byref(h))
        print(rc, h.value, geoloc.geoloc_last_error())
    """)
    env = dict(os.environ, HIP_VISIBLE_DEVICES="-1", ROCR_VISIBLE_DEVICES="-1")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120)
    assert out.returncode == 0, out.stderr
    rc, hv = out.stdout.split()[:2]
    assert int(rc) == geoloc.EDEVICE and hv == "None", out.stdout


def test_subbands_validation_returns_einval():
    """Argument checks of the sub-band split happen before any device call."""
    lib = geoloc.load()
    buf = ctypes.c_void_p(4096)          # never dereferenced: each call fails validation first
    cases = [
        (None, 2, 1600, 16, 64, buf),          # null input
        (buf, 2, 1600, 16, 64, None),          # null output
        (ctypes.c_void_p(4100), 2, 1600, 16, 64, buf),   # misaligned
        (buf, 0, 1600, 16, 64, buf),           # no channels
        (buf, 2, 0, 16, 64, buf),              # no samples
        (buf, 2, 1600, 0, 64, buf),            # no bands
        (buf, 2, 1600, 64, 16, buf),           # too many bands
        (buf, 2, 1601, 16, 64, buf),           # samples not divisible by bands
        (buf, 2, 1600, 16, 0, buf),            # no taps
        (buf, 2, 1600, 16, 129, buf),          # too many taps
        (buf, 2, 1600, 32, 100, buf),          # band table too large
    ]
    for c in cases:
        rc = lib.geoloc_subbands(c[0], c[1], c[2], c[3], c[4], c[5], None)
        assert rc == geoloc.EINVAL, (c, rc, geoloc.geoloc_last_error())


def test_cfar_scale_matches_the_oracle():
    """geoloc_cfar_scale (continued fraction of the incomplete beta, bisection) against the
    oracle's Beta quantile (scipy) to 1e-9, over the window sizes and look counts the
    detection uses; L = 1 also against the exponential closed form N (pfa^(-1/N) - 1)."""
    from oracle import cfar
    for pfa in (1e-2, 1e-3, 2e-3, 1e-6, 1e-9):
        for n_train in (8, 48, 240, 920):
            for looks in (1, 2, 8, 58):
                got = geoloc.geoloc_cfar_scale(pfa, n_train, looks)
                ref = cfar.scale_for_pfa(pfa, n_train, looks)
                assert abs(got - ref) <= 1e-9 * ref, (pfa, n_train, looks, got, ref)
            closed = n_train * (pfa ** (-1.0 / n_train) - 1.0)
            assert abs(geoloc.geoloc_cfar_scale(pfa, n_train, 1) - closed) <= 1e-9 * closed


@pytest.mark.parametrize("args", [(0.0, 10, 1), (1.0, 10, 1), (float("nan"), 10, 1), (1e-3, 0, 1), (1e-3, 10, 0)])
def test_cfar_scale_rejects_bad_arguments(args):
    lib = geoloc.load()
    out = ctypes.c_double(-7.0)
    assert lib.geoloc_cfar_scale(*args, ctypes.byref(out)) == geoloc.EINVAL
    assert out.value == -7.0
    assert lib.geoloc_cfar_scale(1e-3, 10, 1, None) == geoloc.EINVAL


def test_fma_probe_validation_returns_einval():
    """The FP32 FMA probe checks its arguments before any device call."""
    lib = geoloc.load()
    buf = ctypes.c_void_p(4096)          # never dereferenced: each call fails validation first
    n = ctypes.c_int64(0)
    for args in [(0, 100, buf, ctypes.byref(n)), (1 << 21, 100, buf, ctypes.byref(n)), (8, 0, buf, ctypes.byref(n)),
                 (8, 1 << 25, buf, ctypes.byref(n)), (8, 100, None, ctypes.byref(n)), (8, 100, buf, None)]:
        assert lib.geoloc_fma_probe(*args, None) == geoloc.EINVAL, args
