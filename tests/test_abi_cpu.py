"""CPU-only checks of the C ABI library: it loads, exports every function the
header declares, and its host-only logic (schedule, argument checking) is
right.  No compute is launched here."""

import ctypes as C
import math
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2208_05683_amd", "libfps.so")


@pytest.fixture(scope="module")
def B():
    if not os.path.exists(LIB):
        from paper_2208_05683_amd import build as bld

        bld.build()
    from paper_2208_05683_amd import binding

    return binding


def test_exports_every_declared_symbol(B):
    names = B.exported_symbols()
    assert len(names) >= 15
    lib = C.CDLL(LIB)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_header_constants_and_version(B):
    assert B.fps_abi_version() == B.FPS_ABI_VERSION == 2
    assert B.FPS_MAX_S == 31
    assert C.sizeof(B.fps_stats) > 0


def test_schedule_matches_eq6_and_oracle(B):
    import oracle as O

    for m in range(0, 45):
        for s in range(1, 32):
            got = B.fps_schedule(m, s)
            assert got == O.schedule(m, s)
            N = m + 1
            q, b = s, math.ceil(N / s)
            if b >= 2:
                g = 1 if N - q * (b - 1) == 1 else 0
                assert got["n_spgemm"] == q + b - 2 - g  # eq. 5


def test_schedule_rejects_bad_arguments(B):
    with pytest.raises(B.FpsError) as e:
        B.fps_schedule(-1, 3)
    assert e.value.status == B.FPS_ERR_INVALID_ARG
    with pytest.raises(B.FpsError):
        B.fps_schedule(5, 0)


def test_status_strings(B):
    lib = B.library()
    for code in range(0, 7):
        assert lib.fps_status_string(code)
    assert lib.fps_status_string(99) == b"unknown status"


def test_plan_create_rejects_host_side_errors_without_device_work(B):
    lib = B.library()
    h = C.c_void_p()
    coeffs = (C.c_double * 3)(1.0, 1.0, 0.5)
    v = B.fps_csr_view()
    v.n, v.nnz, v.row_ptr, v.col, v.val = 4, 0, 0x1000, None, None  # never dereferenced on these paths
    assert lib.fps_plan_create(C.byref(h), None, coeffs, 2, 2, 1e-12, 0, None) == B.FPS_ERR_INVALID_ARG
    assert lib.fps_plan_create(C.byref(h), C.byref(v), coeffs, -1, 2, 1e-12, 0, None) == B.FPS_ERR_INVALID_ARG
    assert lib.fps_plan_create(C.byref(h), C.byref(v), coeffs, 2, 0, 1e-12, 0, None) == B.FPS_ERR_INVALID_ARG
    assert lib.fps_plan_create(C.byref(h), C.byref(v), coeffs, 2, 32, 1e-12, 0, None) == B.FPS_ERR_INVALID_ARG
    assert lib.fps_plan_create(C.byref(h), C.byref(v), coeffs, 2, 2, float("nan"), 0, None) == B.FPS_ERR_INVALID_ARG
    assert lib.fps_plan_create(C.byref(h), C.byref(v), coeffs, 2, 2, -1.0, 0, None) == B.FPS_ERR_INVALID_ARG
    bad = (C.c_double * 3)(1.0, float("inf"), 0.5)
    assert lib.fps_plan_create(C.byref(h), C.byref(v), bad, 2, 2, 1e-12, 0, None) == B.FPS_ERR_INVALID_ARG
    assert b"coefficient" in lib.fps_last_error()
    v.n = 0
    assert lib.fps_plan_create(C.byref(h), C.byref(v), coeffs, 2, 2, 1e-12, 0, None) == B.FPS_ERR_INVALID_ARG
    assert h.value is None


def test_result_calls_reject_null_plan(B):
    lib = B.library()
    n = C.c_int64()
    assert lib.fps_result_nnz(None, C.byref(n)) == B.FPS_ERR_INVALID_ARG
    assert lib.fps_eval(None, None) == B.FPS_ERR_INVALID_ARG
    lib.fps_plan_destroy(None)
    lib.fps_matrix_destroy(None)


def test_product_path_has_no_oracle_dependency():
    # the package and the library never reference the oracle
    pkg = os.path.join(ROOT, "paper_2208_05683_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f
    with open(LIB, "rb") as f:
        assert b"orc_" not in f.read()


def test_plan_create_ex_rejects_bad_filter_options(B):
    lib = B.library()
    h = C.c_void_p()
    coeffs = (C.c_double * 5)(1.0, 1.0, 0.5, 1.0 / 6, 1.0 / 24)
    v = B.fps_csr_view()
    v.n, v.nnz, v.row_ptr, v.col, v.val = 4, 0, 0x1000, None, None  # never dereferenced on these paths
    o = B.fps_filter_opts()
    assert lib.fps_plan_create_ex(C.byref(h), C.byref(v), coeffs, 4, 2, None, 0, None) == B.FPS_ERR_INVALID_ARG
    o.filter = 7
    assert lib.fps_plan_create_ex(C.byref(h), C.byref(v), coeffs, 4, 2, C.byref(o), 0, None) == B.FPS_ERR_INVALID_ARG
    o.filter = B.FPS_FILTER_ADAPTIVE
    o.eps, o.e_r = 0.0, 0.1
    assert lib.fps_plan_create_ex(C.byref(h), C.byref(v), coeffs, 4, 2, C.byref(o), 0, None) == B.FPS_ERR_INVALID_ARG
    o.eps = 1e-12
    o.e_r = -1.0
    assert lib.fps_plan_create_ex(C.byref(h), C.byref(v), coeffs, 4, 2, C.byref(o), 0, None) == B.FPS_ERR_INVALID_ARG
    assert h.value is None


def test_series_entry_points_reject_bad_arguments_on_the_host(B):
    lib = B.library()
    h = C.c_void_p()
    v = B.fps_csr_view()
    v.n, v.nnz, v.row_ptr, v.col, v.val = 4, 0, 0x1000, None, None  # never dereferenced on these paths
    a = (C.c_double * 8)(*[1.0 / math.factorial(k) for k in range(8)])
    o = B.fps_series_opts()
    o.eps_tol, o.e_r, o.K = 1e-10, 0.1, 10
    assert lib.fps_plan_create_series(C.byref(h), C.byref(v), a, 1, C.byref(o), 0, None) == B.FPS_ERR_INVALID_ARG
    o.eps_tol = 0.0
    assert lib.fps_plan_create_series(C.byref(h), C.byref(v), a, 8, C.byref(o), 0, None) == B.FPS_ERR_INVALID_ARG
    o.eps_tol, o.K = 1e-10, 7
    assert lib.fps_plan_create_series(C.byref(h), C.byref(v), a, 8, C.byref(o), 0, None) == B.FPS_ERR_INVALID_ARG
    o.K = 10
    bad = (C.c_double * 8)(*([1.0] * 7 + [float("nan")]))
    assert lib.fps_plan_create_series(C.byref(h), C.byref(v), bad, 8, C.byref(o), 0, None) == B.FPS_ERR_INVALID_ARG
    assert lib.fps_plan_create_series(C.byref(h), C.byref(v), a, 8, None, 0, None) == B.FPS_ERR_INVALID_ARG
    assert h.value is None
    est = C.c_double()
    assert lib.fps_normest1(C.byref(v), -1, C.byref(est), None, None, 0, None) == B.FPS_ERR_INVALID_ARG
    assert lib.fps_normest1(C.byref(v), 2, None, None, None, 0, None) == B.FPS_ERR_INVALID_ARG
    z = (C.c_double * 4)()
    assert lib.fps_power_norm_bounds(C.byref(v), 3, 3, z, 0, None) == B.FPS_ERR_INVALID_ARG
    assert lib.fps_power_norm_bounds(C.byref(v), 10, -1, z, 0, None) == B.FPS_ERR_INVALID_ARG
    assert lib.fps_plan_series_info(None, None, None, None, None, None) == B.FPS_ERR_INVALID_ARG


def test_binding_shares_torchs_hip_runtime():
    # importing the binding before torch must still leave one HIP runtime in
    # the process (libfps.so binds to the one torch loads)
    import subprocess
    import sys

    code = ("from paper_2208_05683_amd import binding\n"
            "import torch, re\n"
            "m = open('/proc/self/maps').read()\n"
            "print(len(set(re.findall(r'\\S*libamdhip64\\S*', m))))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
