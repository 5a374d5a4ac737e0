"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/pa.h declares, and validates arguments before any device work."""
import ctypes
import os
import re

import pytest

import paper_1703_03676_amd as pa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pa.h")


def declared_functions():
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return sorted(set(re.findall(r"\b(pa_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 15
    raw = ctypes.CDLL(pa.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n
    assert set(names) == set(pa.SIGNATURES)


def test_header_is_plain_c(tmp_path):
    """include/pa.h is a C header of plain types: it compiles as C99 with gcc
    -pedantic -Werror, and every declared entry point can be named from C."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    src = tmp_path / "uses_header.c"
    refs = "\n".join("    (void)&%s;" % n for n in declared_functions())
    src.write_text('#include "pa.h"\nint main(void)\n{\n%s\n    return 0;\n}\n' % refs)
    r = subprocess.run([gcc, "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-I",
                        os.path.join(ROOT, "include"), "-c", str(src), "-o", str(tmp_path / "uses_header.o")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_status_codes_match_header():
    txt = open(HEADER).read()
    for name, val in re.findall(r"(PA_E[A-Z]+|PA_OK)\s*=\s*(-?\d+)", txt):
        assert getattr(pa, name) == int(val)
        assert pa.strerror(int(val)) != "unknown status"


def test_header_constants_match_binding():
    """Every enum value and macro the header defines with a plain number (layouts,
    flags, step modes, statistics paths, limits) that the binding also names has
    the same value there."""
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    consts = dict(re.findall(r"\b(PA_[A-Z_0-9]+)\s*=\s*(-?\d+)", txt))
    consts.update(re.findall(r"#define\s+(PA_[A-Z_0-9]+)\s+\(?(\d+)\)?\s*$", txt, flags=re.M))
    shared = [k for k in consts if hasattr(pa, k)]
    assert {"PA_SPIN_INTERLEAVED", "PA_FLAG_LCG", "PA_STATS_PASS"} <= set(shared)
    for k in shared:
        assert getattr(pa, k) == int(consts[k]), k


def test_workspace_bytes_validation():
    ok = pa.make_params(64, 20000, 1)
    n_bits = pa.workspace_bytes(ok)
    n_int8 = pa.workspace_bytes(pa.make_params(64, 20000, 1, layout="int8"))
    assert 2 * 20000 * 512 < n_bits < n_int8
    assert n_int8 > 2 * 20000 * 4096
    assert pa.workspace_bytes(pa.make_params(64, 20000, 1, mhr=True)) > n_bits
    for bad in (pa.make_params(63, 10, 1), pa.make_params(48, 10, 1), pa.make_params(8, 10, 1),
                pa.make_params(512, 10, 1), pa.make_params(16, 0, 1), pa.make_params(16, 10, 1, capacity=5),
                pa.make_params(16, 10, 1, layout=7)):
        assert pa.workspace_bytes(bad) == 0
    bad_flags = pa.make_params(16, 10, 1)
    for flags in (8, pa.PA_FLAG_HEATBATH | pa.PA_FLAG_LCG):
        bad_flags.flags = flags
        assert pa.workspace_bytes(bad_flags) == 0
    bad_run = pa.make_params(16, 10, 1, run_id=1 << 28)
    assert pa.workspace_bytes(bad_run) == 0
    assert pa.workspace_bytes(pa.make_params(16, 10, 1, run_id=(1 << 28) - 1)) > 0
    assert pa.workspace_bytes(pa.make_params(64, 20000, 1, lcg=True)) == n_bits
    # interleaved store: N site rows of the capacity rounded up to 64 bytes, twice
    n_il = pa.workspace_bytes(pa.make_params(64, 20000, 1, layout="interleaved"))
    assert n_il >= 2 * 4096 * 21504 and n_il >= n_int8
    # the heat-bath update needs no extra device memory
    assert pa.workspace_bytes(pa.make_params(64, 20000, 1, heatbath=True)) == n_bits
    assert pa.workspace_bytes(pa.make_params(64, 20000, 1, heatbath=True, mhr=True)) == \
        pa.workspace_bytes(pa.make_params(64, 20000, 1, mhr=True))
    for L in pa.SUPPORTED_L:
        assert pa.workspace_bytes(pa.make_params(L, 3, 1)) > 0


def test_init_validates_before_device_work():
    lib = pa.lib()
    h = ctypes.c_void_p()
    p = pa.make_params(16, 10, 1)
    need = pa.workspace_bytes(p)
    # NULL workspace, misaligned workspace, too small workspace, invalid params:
    # all rejected on the host before any HIP call.
    assert lib.pa_init(ctypes.byref(p), None, need, None, ctypes.byref(h)) == pa.PA_EINVAL
    assert lib.pa_init(ctypes.byref(p), ctypes.c_void_p(4096 + 8), need, None, ctypes.byref(h)) == pa.PA_EINVAL
    assert lib.pa_init(ctypes.byref(p), ctypes.c_void_p(4096), need - 1, None, ctypes.byref(h)) == pa.PA_ENOMEM
    bad = pa.make_params(17, 10, 1)
    assert lib.pa_init(ctypes.byref(bad), ctypes.c_void_p(4096), 1 << 30, None, ctypes.byref(h)) == pa.PA_EINVAL
    assert lib.pa_init(ctypes.byref(p), ctypes.c_void_p(4096), need, None, None) == pa.PA_EINVAL
    assert not h.value


def test_null_handle():
    lib = pa.lib()
    assert lib.pa_sweep(None, 1) == pa.PA_EINVAL
    assert lib.pa_resample(None, 0.1, None) == pa.PA_EINVAL
    assert lib.pa_observables(None, None) == pa.PA_EINVAL
    assert lib.pa_state(None, None) == pa.PA_EINVAL
    assert lib.pa_set_tie_queue_cap(None, 8) == pa.PA_EINVAL
    assert lib.pa_set_stats_path(None, pa.PA_STATS_EPILOGUE) == pa.PA_EINVAL
    sched = pa.make_schedule(beta_f=1.0, dbeta=0.01, theta=1)
    n = ctypes.c_int32(7)
    assert lib.pa_anneal(None, ctypes.byref(sched), 10, None, None, 0, ctypes.byref(n)) == pa.PA_EINVAL
    assert n.value == 0
    assert lib.pa_free(None) == pa.PA_OK
    assert lib.pa_last_error(None) == b""


def test_binding_refuses_to_run_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        pa.Run(16, 10, seed=1)


def test_observables_static_validates_before_device_work():
    lib = pa.lib()
    o = pa.Obs()
    h = pa.PA_STATIC_MAX_R
    dev = ctypes.c_void_p(4096)  # never dereferenced: every case fails validation first
    assert lib.pa_observables_static(64, 0, dev, dev, 0.0, 0.0, 0.0, None, ctypes.byref(o)) == pa.PA_EINVAL
    assert lib.pa_observables_static(64, h + 1, dev, dev, 0.0, 0.0, 0.0, None, ctypes.byref(o)) == pa.PA_EINVAL
    for L in (8, 48, 63, 512):
        assert lib.pa_observables_static(L, 10, dev, dev, 0.0, 0.0, 0.0, None, ctypes.byref(o)) == pa.PA_EINVAL
    assert lib.pa_observables_static(64, 10, None, dev, 0.0, 0.0, 0.0, None, ctypes.byref(o)) == pa.PA_EINVAL
    assert lib.pa_observables_static(64, 10, dev, None, 0.0, 0.0, 0.0, None, ctypes.byref(o)) == pa.PA_EINVAL
    assert lib.pa_observables_static(64, 10, dev, dev, 0.0, 0.0, 0.0, None, None) == pa.PA_EINVAL
    assert lib.pa_observables_static(64, 10, dev, dev, float("nan"), 0.0, 0.0, None, ctypes.byref(o)) == pa.PA_EINVAL
    assert lib.pa_static_scratch_bytes() < 1 << 20
