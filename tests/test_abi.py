"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_1008_0502_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "salprior.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsalprior.so is not built (run python -m paper_1008_0502_amd.build)")
    return _lib.load()


def test_header_symbols_are_exported(lib):
    names = header_functions()
    assert {"saliency_forward", "saliency_backward", "prior_update", "mrf_weights"} <= set(names)
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), f"{n} declared in salprior.h but not exported"
    declared = {s[0] for s in _lib.SIGNATURES}
    assert set(names) == declared, "binding signature table out of sync with the header"


def test_default_params_match_header(lib):
    p = _lib.sp_params()
    lib.sp_default_params(ctypes.byref(p))
    assert p.depth == 0 and p.n_centers == 2 and list(p.centers)[:2] == [1, 2]
    assert p.n_deltas == 2 and list(p.deltas)[:2] == [2, 3]
    assert list(p.weights) == [1.0] * 8
    assert p.q == 1e-3 and p.r == 1e-1
    assert p.eps == pytest.approx(1e-4) and p.border == 1 and p.lm_block == 8
    assert p.flat_tol == pytest.approx(1e-5) and p.gabor_radius == 6


def test_struct_layout_matches_c_compiler(tmp_path):
    # compile a probe against the public header with the host C compiler and compare
    # every field offset with the ctypes mirror used by the binding
    fields = [f for f, _ in _lib.sp_params._fields_]
    cfields = [f.rstrip("_") for f in fields]
    gfields = [f for f, _ in _lib.sp_geometry._fields_]
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "salprior.h"', "int main(void){",
           'printf("%zu %zu\\n", sizeof(sp_params), sizeof(sp_geometry));']
    src += [f'printf("%zu\\n", offsetof(sp_params, {f}));' for f in cfields]
    src += [f'printf("%zu\\n", offsetof(sp_geometry, {f}));' for f in gfields]
    src += ["return 0;}"]
    c = tmp_path / "probe.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "probe"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    vals = [int(v) for v in out]
    assert vals[0] == ctypes.sizeof(_lib.sp_params) and vals[1] == ctypes.sizeof(_lib.sp_geometry)
    offs = vals[2:]
    for i, f in enumerate(fields):
        assert offs[i] == getattr(_lib.sp_params, f).offset, f
    for j, f in enumerate(gfields):
        assert offs[len(fields) + j] == getattr(_lib.sp_geometry, f).offset, f


def _create(lib, p, H=120, W=160):
    h = ctypes.c_void_p()
    rc = lib.sp_create(ctypes.byref(p), H, W, None, ctypes.byref(h))
    return rc, lib.sp_last_error().decode(), h


@pytest.mark.parametrize("field,value,code", [
    ("lm_block", 4, _lib.SP_EINVAL),
    ("gabor_radius", 9, _lib.SP_EINVAL),
    ("gabor_radius", 0, _lib.SP_EINVAL),
    ("n_centers", 0, _lib.SP_EINVAL),
    ("n_deltas", 5, _lib.SP_EINVAL),
    ("eps", 0.0, _lib.SP_EINVAL),
    ("eps", 0.6, _lib.SP_EINVAL),
    ("q", float("nan"), _lib.SP_EINVAL),
    ("r", -1.0, _lib.SP_EINVAL),
    ("border", -1, _lib.SP_EINVAL),
    ("lambda_", float("inf"), _lib.SP_EINVAL),
    ("flat_tol", -1.0, _lib.SP_EINVAL),
    ("record_tape", -3, _lib.SP_EINVAL),
    ("depth", 2, _lib.SP_ESHAPE),          # no pair (c, c + delta) fits depth 2
    ("depth", 13, _lib.SP_ESHAPE),
])
def test_create_rejects_bad_params(lib, field, value, code):
    p = _lib.sp_params()
    lib.sp_default_params(ctypes.byref(p))
    setattr(p, field, value)
    rc, msg, h = _create(lib, p)
    assert rc == code, msg
    assert msg and not h.value


def test_create_rejects_bad_shapes_and_nulls(lib):
    p = _lib.sp_params()
    lib.sp_default_params(ctypes.byref(p))
    for H, W in [(0, 10), (5, 0), (3, 3), (70000, 8), (20000, 20000)]:
        rc, msg, _ = _create(lib, p, H, W)
        assert rc == _lib.SP_ESHAPE, (H, W, msg)
    p.q = 0.0
    p.r = 0.0
    assert _create(lib, p)[0] == _lib.SP_EINVAL
    lib.sp_default_params(ctypes.byref(p))
    p.centers[0], p.centers[1] = 1, 4          # centre span 3 octaves
    p.deltas[0], p.deltas[1] = 1, 2
    p.depth = 7
    assert _create(lib, p, 480, 640)[0] == _lib.SP_ESHAPE
    h = ctypes.c_void_p()
    assert lib.sp_create(None, 10, 10, None, ctypes.byref(h)) == _lib.SP_EINVAL
    assert lib.saliency_forward(None, None, None, None, None) == _lib.SP_EINVAL
    assert lib.prior_update(None, None, None, None) == _lib.SP_EINVAL
    assert lib.mrf_weights(None, None, None, None, None, None) == _lib.SP_EINVAL
    assert lib.saliency_backward(None, None, 1, None, None, None) == _lib.SP_EINVAL
    assert lib.sp_destroy(None) == _lib.SP_OK
    assert lib.sp_last_error() == b""
    hb = ctypes.c_void_p()
    Hs = (ctypes.c_int32 * 2)(120, 240)
    Ws = (ctypes.c_int32 * 2)(160, 320)
    lib.sp_default_params(ctypes.byref(p))
    assert lib.sp_batch_create(ctypes.byref(p), 0, Hs, Ws, 0, None, ctypes.byref(hb)) == _lib.SP_EINVAL
    assert lib.sp_batch_create(ctypes.byref(p), 2, Hs, Ws, 8, None, ctypes.byref(hb)) == _lib.SP_EINVAL
    p.record_tape = -1
    assert lib.sp_batch_create(ctypes.byref(p), 2, Hs, Ws, 0, None, ctypes.byref(hb)) == _lib.SP_EINVAL
    assert lib.sp_batch_backward(None, None, 1, None, None, None) == _lib.SP_EINVAL
    assert lib.sp_batch_mse_mask_loss(None, None, 1, None, None) == _lib.SP_EINVAL
    assert lib.sp_batch_set_weights(None, None, 1e-3, 1e-1) == _lib.SP_EINVAL
    assert lib.sp_batch_step_index(None) == -1 and lib.sp_batch_tape_generation(None) == -1
    tabs = (ctypes.c_void_p * 2)(None, None)
    assert lib.sp_batch_steps(None, 2, tabs) == _lib.SP_EINVAL


def test_product_path_has_no_cpu_fallback():
    # the binding raises when the library is missing instead of computing elsewhere
    import importlib
    src = open(os.path.join(ROOT, "paper_1008_0502_amd", "api.py")).read()
    assert "oracle" not in src and "numpy" not in src
    with pytest.raises(RuntimeError):
        saved = _lib._LIB
        try:
            _lib._LIB = None
            _lib.load(os.path.join(ROOT, "does_not_exist.so"))
        finally:
            _lib._LIB = saved


def test_noalloc_rejects_frames_beyond_its_scratch(lib):
    # sized before any device call: a 4K frame needs more than the array holds
    p = _lib.sp_params()
    lib.sp_default_params(ctypes.byref(p))
    rc = lib.sp_saliency_noalloc(ctypes.byref(p), 2160, 3840, 1, None, 1, None, None)
    assert rc == _lib.SP_ESHAPE
    msg = lib.sp_last_error().decode()
    assert "needs" in msg and str(64 << 20) in msg
    assert lib.sp_saliency_noalloc(ctypes.byref(p), 480, 640, None, None, 1, None, None) == _lib.SP_EINVAL
    assert lib.sp_saliency_noalloc(None, 480, 640, 1, None, 1, None, None) == _lib.SP_EINVAL
