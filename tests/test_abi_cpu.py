"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/yastn.h declares, and rejects malformed problems with
the same status class as the oracle's validation."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2405_12196_amd as Y
import workloads as W
from tests.helpers import random_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "yastn.h")).read()
    return sorted(set(re.findall(r"\b(yastn_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = Y.lib()
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), f"{n} not exported"
    assert set(names) == set(Y.EXPORTS)
    assert L.yastn_abi_version() == 1
    assert L.yastn_status_string(0) == b"YASTN_OK"
    assert L.yastn_status_string(4) == b"YASTN_ERR_SIGNATURE"
    assert L.yastn_norm_workspace() > 0


def _status(a, b, xa, xb, **kw):
    try:
        Y.plan([(a, b, xa, xb)], stream=0, **kw)
    except Y.YastnError as e:
        return e.status
    return "OK"


def _oracle_status(a, b, xa, xb):
    try:
        oracle.validate_pair(a, b, xa, xb)
    except oracle.OracleError as e:
        return e.status
    return "OK"


def _cases():
    (p,) = W.u1_d18()
    a, b = p.a, p.b
    out = [("axes length", a, b, (2, 3), (0,)), ("axes repeated", a, b, (2, 2), (0, 1)),
           ("axes range", a, b, (2, 7), (0, 1)), ("equal signature", a, b, (0, 1), (0, 1))]
    bad = a.copy(); bad.charges[3, 0, 0] += 1
    out.append(("charge", bad, b, (2, 3), (0, 1)))
    bad = a.copy(); bad.shapes[0, 0] = 0
    out.append(("dim zero", bad, b, (2, 3), (0, 1)))
    bad = a.copy(); bad.charges[1] = bad.charges[0]; bad.shapes[1] = bad.shapes[0]
    out.append(("duplicate", bad, b, (2, 3), (0, 1)))
    bad = b.copy(); bad.sym_mod = (2,)
    out.append(("symmetry", a, bad, (2, 3), (0, 1)))
    bad = a.copy(); bad.offsets[1] = bad.offsets[0]
    out.append(("overlap", bad, b, (2, 3), (0, 1)))
    bad = a.copy(); bad.sig = bad.sig.copy(); bad.sig[0] = 2
    out.append(("signature value", bad, b, (2, 3), (0, 1)))
    legs = [W._u1_leg(s, [(-1, 2), (0, 3), (1, 2)]) for s in (1, -1)]
    x = W.rand(legs, (0,), (0,), 1)
    y = W.rand([W._u1_leg(s, [(-1, 2), (0, 4), (1, 2)]) for s in (1, -1)], (0,), (0,), 2)
    out.append(("contracted dim", x, y, (1,), (0,)))
    bad = a.copy(); bad.shapes = bad.shapes.copy(); bad.shapes[5, 1] += 1
    out.append(("two dims on a leg", bad, b, (2, 3), (0, 1)))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_status_class_matches_oracle(case):
    name, a, b, xa, xb = case
    want = _oracle_status(a, b, xa, xb)
    assert want != "OK"
    assert _status(a, b, xa, xb) == want


def test_valid_problem_without_gpu_is_hip_error_or_ok():
    # validation passes; without a device the join cannot run
    import torch
    (p,) = W.u1_d18()
    st = _status(p.a, p.b, p.axes_a, p.axes_b)
    if torch.cuda.is_available():
        assert st == "OK"
    else:
        assert st == "ERR_HIP"


@pytest.mark.parametrize("seed", range(20))
def test_random_valid_problems_pass_host_validation(seed):
    a, b, xa, xb = random_problem(seed + 300, ["U1", "Z2", "U1xZ2"][seed % 3], keep=0.8, shuffle=seed % 2 == 0)
    assert _oracle_status(a, b, xa, xb) == "OK"
    assert _status(a, b, xa, xb) in ("OK", "ERR_HIP")


def test_bad_options_rejected():
    (p,) = W.u1_d18()
    with pytest.raises(Y.YastnError) as e:
        Y.plan([(p.a, p.b, p.axes_a, p.axes_b)], precision="f64", in_dtype=Y.DTYPE_F32, stream=0)
    assert e.value.status == "ERR_ARG"
    with pytest.raises(Y.YastnError) as e:
        Y.plan([(p.a, p.b, p.axes_a, p.axes_b)], tile_rows=48, stream=0)
    assert e.value.status == "ERR_ARG"


def test_null_arguments_rejected():
    L = Y.lib()
    h = ctypes.c_void_p()
    assert L.yastn_plan(None, 1, None, None, ctypes.byref(h)) == 1
    assert L.yastn_plan_workspace(None, None) == 1
    assert L.yastn_norm(None, 10, 0, None, None, None) == 1
    L.yastn_free(None)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and says so,
    before touching any device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_variant_count_matches_header():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with open(os.path.join(root, "include", "yastn.h")) as f:
        n = int(re.search(r"#define YASTN_NUM_VARIANTS (\d+)", f.read()).group(1))
    assert Y.NUM_VARIANTS == n


def test_complex_and_swap_gate_host_errors():
    """Errors the host finds before any device work: complex operands whose
    real form would exceed the rank limit, unknown conj flags, swap-gate legs
    out of range, a fermionic mask entry other than 0 / 1, C128 for yastn_norm."""
    from workloads import Leg
    v = Leg(1, ((0,), (1,)), (1, 2))
    big = W.rand_complex([v] * 4 + [v.conj()] * 4, (0,), (2,), 1)   # rank 8: no room for (re, im)
    small = W.rand_complex([v, v.conj()], (0,), (2,), 2)
    with pytest.raises(Y.YastnError) as e:
        Y.ZPlan([(big, small, (0,), (1,))], stream=0)
    assert e.value.status == "ERR_ARG"
    with pytest.raises(Y.YastnError) as e:
        Y.ZPlan([(small, small, (1,), (0,))], conj=4, stream=0)
    assert e.value.status == "ERR_ARG"
    with pytest.raises(Y.YastnError) as e:
        Y.SwapGate(small, (0,), (2,), (1,))
    assert e.value.status == "ERR_ARG"
    with pytest.raises(Y.YastnError) as e:
        Y.SwapGate(small, (0,), (1,), (2,))
    assert e.value.status == "ERR_ARG"
    assert Y.lib().yastn_norm(None, 10, Y.DTYPE_C128, None, None, None) == 1


def test_tuning_store_file_format(tmp_path):
    """The tuning store's file round-trips on the host; files that are not
    tuning files, were made for another variant count, or hold an entry with
    a variant out of range are rejected and leave the store as it was."""
    Y.tune_clear()
    p = tmp_path / "tune.json"
    Y.tune_save(str(p))
    txt = p.read_text()
    assert '"format": "yastn-tuning"' in txt and f'"variants": {Y.NUM_VARIANTS}' in txt
    assert Y.tune_load(str(p)) == 0
    ms = ", ".join(["0.5"] * Y.NUM_VARIANTS)
    good = ('{"format": "yastn-tuning", "version": 1, "variants": %d,\n "entries": [\n'
            '  {"key": "%s", "arch": "gfx950", "variant": 21, "ms": [%s]}\n ]}\n'
            % (Y.NUM_VARIANTS, "0123456789abcdef" * 2, ms))
    q = tmp_path / "one.json"
    q.write_text(good)
    assert Y.tune_load(str(q)) == 1
    r = tmp_path / "again.json"
    Y.tune_save(str(r))
    assert "0123456789abcdef0123456789abcdef" in r.read_text() and '"variant": 21' in r.read_text()
    for bad in ('{"something": 1}',
                good.replace('"variants": %d' % Y.NUM_VARIANTS, '"variants": 7'),
                good.replace('"variant": 21', '"variant": 99'),
                good.replace("0123456789abcdef" * 2, "xyz")):
        q.write_text(bad)
        with pytest.raises(Y.YastnError) as e:
            Y.tune_load(str(q))
        assert e.value.status == "ERR_ARG"
    with pytest.raises(Y.YastnError):
        Y.tune_load(str(tmp_path / "missing.json"))
    Y.tune_clear()
