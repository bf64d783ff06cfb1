"""Host-only checks of the C ABI (no device calls).

* libdpt.so loads and exports every function ``include/dpt.h`` declares;
* the ctypes mirrors of the structs have the C layout (sizeof / offsetof from a
  probe compiled with the system C compiler against the header);
* ``dpt_validate`` rejects bad arguments without touching a device.
"""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from paper_2002_12872_amd import dpt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(dpt_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    lib = dpt.load_library()
    names = declared_functions()
    assert len(names) >= 11
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(dpt._FUNCS)


def test_struct_layout_matches_header(tmp_path):
    probe = tmp_path / "probe.c"
    classes = {"dpt_problem": dpt.Problem, "dpt_options": dpt.Options, "dpt_result": dpt.Result,
               "dpt_profile": dpt.Profile, "dpt_serve_config": dpt.ServeConfig,
               "dpt_serve_times": dpt.ServeTimes, "dpt_serve_stats": dpt.ServeStats}
    fields = {k: [f[0] for f in c._fields_] for k, c in classes.items()}
    cname = {"lam": "lambda"}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "dpt.h"', "int main(void){"]
    for st, fs in fields.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (st, st))
        for f in fs:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (st, f, st, cname.get(f, f)))
    lines.append("return 0;}")
    probe.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(probe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                      check=True).stdout.splitlines())
    for st, cls in classes.items():
        assert int(out[st]) == ctypes.sizeof(cls), st
        for f in fields[st]:
            assert int(out["%s.%s" % (st, f)]) == getattr(cls, f).offset, (st, f)


def test_status_strings():
    for code in (0, 1, 2, 3, 4, -1, -2, -3, -4):
        s = dpt.dpt_status_str(code)
        assert s.startswith("DPT_")
    assert dpt.dpt_status_str(99) == "unknown status"


def test_options_default():
    o = dpt.dpt_options_default()
    assert o.tol == 1e-6 and o.max_iter == 200 and o.precision == dpt.DPT_FP32
    assert o.stall_ratio == 0.5 and o.stall_patience == 2 and o.check_every == 1
    assert o.blowup == 1e6 and o.fp64_final_tol == 0.0
    assert o.stop_rule == dpt.DPT_STOP_DELTA and o.reserved == 0


def _spec(n=4, theta=None, delta=None, lam=0.1):
    theta = np.arange(n, dtype=np.float64) if theta is None else theta
    delta = np.zeros((n, n)) if delta is None else delta
    return dpt.ProblemSpec(theta, delta, lam, stream=0)


def test_validate_accepts_good_problem():
    assert dpt.dpt_validate(_spec()) == dpt.DPT_OK
    assert dpt.dpt_validate(_spec(), dpt.options(precision=dpt.DPT_BF16_FP32)) == dpt.DPT_OK


@pytest.mark.parametrize("mutate", [
    lambda p: setattr(p.struct, "n", 0),
    lambda p: setattr(p.struct, "theta", None),
    lambda p: setattr(p.struct, "delta", None),
    lambda p: setattr(p.struct, "format", 7),
    lambda p: setattr(p.struct, "dtype", 9),
    lambda p: setattr(p.struct, "mem", 5),
    lambda p: setattr(p.struct, "reserved", 1),
    lambda p: setattr(p.struct, "lam", float("nan")),
    lambda p: setattr(p.struct, "lam", float("inf")),
])
def test_validate_rejects_bad_problem(mutate):
    p = _spec()
    mutate(p)
    assert dpt.dpt_validate(p) == dpt.DPT_EINVAL


def test_validate_rejects_degenerate_theta():
    # unperturbed eigenvalues must be simple (Sec. II.B)
    p = _spec(theta=np.array([0.0, 1.0, 2.0, 1.0]))
    assert dpt.dpt_validate(p) == dpt.DPT_EINVAL
    p = _spec(theta=np.array([0.0, np.nan, 2.0, 3.0]))
    assert dpt.dpt_validate(p) == dpt.DPT_EINVAL


@pytest.mark.parametrize("bad", ["indptr0", "decreasing", "col_range", "unsorted", "dup", "nnz"])
def test_validate_rejects_bad_csr(bad):
    indptr = np.array([0, 2, 3, 5], np.int64)
    indices = np.array([1, 2, 0, 0, 1], np.int32)
    values = np.ones(5)
    if bad == "indptr0":
        indptr = indptr + 1
    elif bad == "decreasing":
        indptr = np.array([0, 3, 2, 5], np.int64)
    elif bad == "col_range":
        indices = np.array([1, 3, 0, 0, 1], np.int32)
    elif bad == "unsorted":
        indices = np.array([2, 1, 0, 0, 1], np.int32)
    elif bad == "dup":
        indices = np.array([1, 1, 0, 0, 1], np.int32)
    p = dpt.ProblemSpec(np.arange(3.0), (indptr, indices, values), 0.1, stream=0)
    if bad == "nnz":
        p.struct.nnz = 4
    assert dpt.dpt_validate(p) == dpt.DPT_EINVAL
    good = dpt.ProblemSpec(np.arange(3.0), (np.array([0, 2, 3, 5], np.int64),
                                            np.array([1, 2, 0, 0, 1], np.int32), values), 0.1, stream=0)
    assert dpt.dpt_validate(good) == dpt.DPT_OK


@pytest.mark.parametrize("field,value", [
    ("tol", 0.0), ("tol", -1.0), ("tol", float("nan")), ("max_iter", -1), ("precision", 5),
    ("fp64_final_tol", -1.0), ("stall_ratio", 1.5), ("stall_patience", 0), ("check_every", 0),
    ("blowup", 0.0), ("stop_rule", 3), ("reserved", 1), ("ramp_alpha", 1.0), ("ramp_alpha", -0.5),
    ("ramp_alpha", float("nan")),
])
def test_validate_rejects_bad_options(field, value):
    o = dpt.options()
    setattr(o, field, value)
    assert dpt.dpt_validate(_spec(), o) == dpt.DPT_EINVAL


@pytest.mark.parametrize("precision,fp64_final_tol,check_every,ok", [
    (1, 0.0, 1, True), (0, 0.0, 1, True), (2, 0.0, 1, True), (3, 0.0, 1, False), (4, 0.0, 1, False),
    (2, 1e-10, 1, False), (1, 0.0, 2, False)])
def test_per_row_rule_only_with_its_precisions(precision, fp64_final_tol, check_every, ok):
    o = dpt.options(precision=precision, fp64_final_tol=fp64_final_tol, check_every=check_every,
                    stop_rule=dpt.DPT_STOP_ROW)
    assert dpt.dpt_validate(_spec(), o) == (dpt.DPT_OK if ok else dpt.DPT_EINVAL)


def test_init_rejects_invalid_before_touching_device():
    p = _spec(theta=np.array([0.0, 0.0, 1.0, 2.0]))
    with pytest.raises(dpt.DptError) as ei:
        dpt.dpt_init(p)
    assert ei.value.code == dpt.DPT_EINVAL


def test_missing_library_fails_loudly():
    """No fallback: without the built library the binding raises at load time."""
    code = ("from paper_2002_12872_amd import dpt\n"
            "try:\n"
            "    dpt.load_library('/nonexistent/libdpt.so')\n"
            "except ImportError as e:\n"
            "    print('raised', e)\n")
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert p.returncode == 0 and p.stdout.startswith("raised"), p.stdout + p.stderr


@pytest.mark.parametrize("kw", [dict(budget_bytes=0), dict(max_slots=0), dict(max_slots=1025),
                                dict(grid_blocks=-1), dict(autotune=2), dict(autotune=-4)])
def test_serve_open_rejects_bad_config_before_touching_device(kw):
    """Config checks come before any runtime call (autotune: 1 tunes, 0 takes the
    defaults, -1 / -2 / -3 force one tile shape; nothing else)."""
    args = dict(budget_bytes=1 << 20, max_slots=4, use_graph=1, grid_blocks=0, autotune=0)
    args.update(kw)
    cfg = dpt.ServeConfig(args["budget_bytes"], args["max_slots"], args["use_graph"], args["grid_blocks"],
                          args["autotune"], None)
    h = ctypes.c_void_p()
    assert dpt.load_library().dpt_serve_open(ctypes.byref(h), ctypes.byref(cfg)) == dpt.DPT_EINVAL
    assert h.value is None
