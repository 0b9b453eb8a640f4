"""Host-side checks of the C ABI: the library loads, exports every function
declared in include/randutv.h, and validates arguments before touching the
GPU (LAPACK-style -i statuses).  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "randutv.h")
LIB = os.path.join(ROOT, "paper_1703_00998_amd", "librandutv.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(randutv_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_1703_00998_amd import binding
    return binding.lib()


def test_header_declares_expected_entry_points():
    names = _declared()
    for n in ["randutv_factor", "randutv_workspace_size", "randutv_g_cols",
              "randutv_random_steps", "randutv_gemm", "randutv_panel_qr",
              "randutv_small_svd", "randutv_strerror"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_names_match_header(lib):
    from paper_1703_00998_amd import binding
    assert set(binding.EXPORTS) <= set(_declared())


def test_step_counts(lib):
    # Figure randUTV: s = min(ceil(m/b), ceil(n/b)); randomized iff I3, J3 nonempty.
    assert lib.randutv_random_steps(500, 500, 32) == 15
    assert lib.randutv_g_cols(500, 500, 32) == 480
    assert lib.randutv_g_cols(8000, 8000, 256) == 7936
    assert lib.randutv_random_steps(4000, 4000, 128) == 31
    assert lib.randutv_random_steps(50, 40, 64) == 0
    assert lib.randutv_random_steps(20000, 5000, 128) == 39
    assert lib.randutv_random_steps(0, 5, 2) == -1
    # Over-sampling: b + p columns per randomized step.
    assert lib.randutv_g_cols_p(500, 500, 32, 0) == 480
    assert lib.randutv_g_cols_p(500, 500, 32, 5) == 15 * 37
    assert lib.randutv_g_cols_p(500, 500, 32, -1) == -1


def test_workspace_and_argument_validation(lib):
    sz = ctypes.c_size_t(0)
    assert lib.randutv_workspace_size(100, 80, 16, 1, 0, 3, ctypes.byref(sz)) == 0
    assert sz.value > 0
    assert lib.randutv_workspace_size(80, 100, 16, 1, 0, 3, ctypes.byref(sz)) == 0  # wide input
    assert lib.randutv_workspace_size(100, 80, 0, 1, 0, 3, ctypes.byref(sz)) == -3
    assert lib.randutv_workspace_size(100, 80, 16, -1, 0, 3, ctypes.byref(sz)) == -4
    assert lib.randutv_workspace_size(100, 80, 16, 1, 7, 3, ctypes.byref(sz)) == -5
    # RANDUTV_ECON_U (4) only together with RANDUTV_FORM_U (1)
    assert lib.randutv_workspace_size(100, 80, 16, 1, 0, 4, ctypes.byref(sz)) == -6
    assert lib.randutv_workspace_size(100, 80, 16, 1, 0, 5, ctypes.byref(sz)) == 0
    assert lib.randutv_workspace_size(100, 80, 16, 1, 0, 11, ctypes.byref(sz)) == 0  # ONE_STREAM
    assert lib.randutv_workspace_size(100, 80, 16, 1, 0, 16, ctypes.byref(sz)) == -6
    vp = ctypes.c_void_p
    null = vp(0)
    fake = vp(1 << 20)  # never dereferenced: validation fails first
    args = dict(m=100, n=80, b=16, q=1, T=fake, ldt=100, G=fake, ldg=100, U=null, ldu=100,
                V=null, ldv=80, k_stop=0, tol=0.0, prec=0, flags=0, work=null, wb=0,
                k=None, st=null)

    def call(**kw):
        a = dict(args, **kw)
        return lib.randutv_factor(a["m"], a["n"], a["b"], a["q"], a["T"], a["ldt"], a["G"],
                                  a["ldg"], a["U"], a["ldu"], a["V"], a["ldv"], a["k_stop"],
                                  a["tol"], a["prec"], a["flags"], a["work"], a["wb"],
                                  a["k"], a["st"])
    assert call(m=0) == -1
    assert call(m=50, work=null) == -12  # m < n accepted (wide last step); then the work check
    assert call(b=0) == -2
    assert call(b=1000) == -2
    assert call(q=-1) == -3
    assert call(T=null) == -4
    assert call(ldt=99) == -4
    assert call(G=null) == -5
    assert call(ldg=10) == -5
    assert call(flags=1) == -6         # U requested but NULL
    assert call(flags=2) == -7
    assert call(prec=5) == -10
    assert call(flags=16) == -11
    assert call(flags=4) == -11        # ECON_U without FORM_U
    assert call() == -12               # no workspace
    assert call(work=vp(4096 + 8)) == -12   # misaligned
    assert call(work=vp(4096), wb=16) == -901
    assert lib.randutv_strerror(-900) == b"unsupported case"


def test_noalloc_entry_point_validates(lib):
    """randutv_factor_noalloc checks its arguments, and the size limit of its
    static workspace, before it touches the device."""
    vp = ctypes.c_void_p
    null = vp(0)
    fake = vp(1 << 20)

    def call(m=100, n=80, b=16, q=1, T=fake, ldt=100, G=fake, U=null, V=null, prec=0, flags=0):
        return lib.randutv_factor_noalloc(m, n, b, q, T, ldt, G, m, U, m, V, n, 0, 0.0, prec,
                                          flags, None, null)
    assert call(m=0) == -1
    assert call(b=0) == -2
    assert call(q=-1) == -3
    assert call(T=null) == -4
    assert call(ldt=50) == -4
    assert call(G=null) == -5
    assert call(flags=1) == -6
    assert call(flags=2) == -7
    assert call(prec=5) == -10
    assert call(flags=16) == -11
    # 4000 x 4000, b = 256 with U and V needs more than the 128 MiB array.
    assert call(m=4000, n=4000, b=256, ldt=4000, U=fake, V=fake, flags=3) == -901


def test_oversampled_entry_points_validate(lib):
    sz = ctypes.c_size_t(0)
    sz0 = ctypes.c_size_t(0)
    assert lib.randutv_workspace_size_p(100, 80, 16, 0, 1, 0, 3, ctypes.byref(sz)) == 0
    assert lib.randutv_workspace_size(100, 80, 16, 1, 0, 3, ctypes.byref(sz0)) == 0
    assert sz.value == sz0.value           # p = 0 is the plain layout
    assert lib.randutv_workspace_size_p(100, 80, 16, 8, 1, 0, 3, ctypes.byref(sz)) == 0
    assert sz.value > sz0.value
    assert lib.randutv_workspace_size_p(100, 80, 16, -1, 1, 0, 3, ctypes.byref(sz)) == -4
    assert lib.randutv_workspace_size_p(100, 80, 250, 7, 1, 0, 3, ctypes.byref(sz)) == -4
    assert lib.randutv_workspace_size_p(100, 80, 16, 4, -1, 0, 3, ctypes.byref(sz)) == -5
    vp = ctypes.c_void_p
    null = vp(0)
    fake = vp(1 << 20)  # never dereferenced: validation fails first

    def call(p=4, b=16, G=fake, ldg=100, work=null, wb=0):
        return lib.randutv_factor_p(100, 80, b, p, 1, fake, 100, G, ldg, null, 100, null, 80,
                                    0, 0.0, 0, 0, work, wb, None, null)
    assert call(p=-1) == -13
    assert call(b=250, p=7) == -13
    assert call(G=null) == -5
    assert call() == -12
    assert call(work=vp(4096), wb=16) == -901


def test_gemm_and_panel_validation(lib):
    vp = ctypes.c_void_p
    f = vp(1 << 20)
    assert lib.randutv_gemm(9, 0, 0, 4, 4, 4, 1.0, f, 4, f, 4, 0.0, f, 4, vp(0), 0, vp(0)) == -1
    assert lib.randutv_gemm(0, 0, 0, 4, 4, 4, 1.0, f, 3, f, 4, 0.0, f, 4, vp(0), 0, vp(0)) == -8
    assert lib.randutv_gemm(0, 1, 0, 4, 4, 5, 1.0, f, 4, f, 5, 0.0, f, 4, vp(0), 0, vp(0)) == -8
    assert lib.randutv_gemm(0, 0, 0, 4, 4, 4, 1.0, f, 4, f, 4, 0.0, f, 3, vp(0), 0, vp(0)) == -13
    assert lib.randutv_panel_qr(10, 20, f, 10, f, f, 20, None, f, 1 << 30, vp(0)) == -2
    assert lib.randutv_panel_qr(100, 300, f, 100, f, f, 300, None, f, 1 << 30, vp(0)) == -2
    assert lib.randutv_panel_qr(100, 8, f, 99, f, f, 8, None, f, 1 << 30, vp(0)) == -3
    assert lib.randutv_panel_qr(100, 8, f, 100, f, f, 8, None, f, 16, vp(0)) == -9
    assert lib.randutv_panel_work_size(100, 0) == 0
    assert lib.randutv_panel_work_size(10, 20) == 0
    assert lib.randutv_panel_work_size(8000, 256) > 8000 * 256 * 8


def test_rsvd_entry_points_validate(lib):
    sz = ctypes.c_size_t(0)
    assert lib.randutv_rsvd_workspace_size(300, 200, 20, 5, 1, 0, ctypes.byref(sz)) == 0
    assert sz.value > 0
    assert lib.randutv_rsvd_workspace_size(300, 200, 0, 5, 1, 0, ctypes.byref(sz)) == -3
    assert lib.randutv_rsvd_workspace_size(300, 200, 20, -1, 1, 0, ctypes.byref(sz)) == -4
    assert lib.randutv_rsvd_workspace_size(300, 200, 190, 20, 1, 0, ctypes.byref(sz)) == -4
    assert lib.randutv_rsvd_workspace_size(300, 200, 250, 10, 1, 0, ctypes.byref(sz)) == -4
    assert lib.randutv_rsvd_workspace_size(300, 200, 20, 5, 17, 0, ctypes.byref(sz)) == -5
    assert lib.randutv_rsvd_workspace_size(300, 200, 20, 5, 1, 9, ctypes.byref(sz)) == -15
    vp = ctypes.c_void_p
    null = vp(0)
    fake = vp(1 << 20)  # never dereferenced: validation fails first

    def call(A=fake, lda=300, G=fake, ldg=300, U=fake, ldu=300, D=fake, V=fake, ldv=200,
             work=null, wb=0):
        return lib.randutv_rsvd(300, 200, 20, 5, 1, A, lda, G, ldg, U, ldu, D, V, ldv, 0,
                                work, wb, None, null)
    assert call(A=null) == -6
    assert call(lda=299) == -6
    assert call(G=null) == -8
    assert call(U=null) == -10
    assert call(D=null) == -12
    assert call(ldv=199) == -13
    assert call() == -16
    assert call(work=vp(4096), wb=16) == -901


def test_lower_entry_points_validate(lib):
    sz = ctypes.c_size_t(0)
    assert lib.randutv_workspace_size_lower(100, 80, 16, 1, 0, 3, ctypes.byref(sz)) == 0
    s0 = ctypes.c_size_t(0)
    assert lib.randutv_workspace_size(80, 100, 16, 1, 0, 3, ctypes.byref(s0)) == 0
    assert sz.value >= s0.value + 100 * 80 * 8     # A^T plus the transposed problem's workspace
    assert lib.randutv_workspace_size_lower(100, 80, 0, 1, 0, 3, ctypes.byref(sz)) == -3
    vp = ctypes.c_void_p
    null = vp(0)
    fake = vp(1 << 20)  # never dereferenced: validation fails first

    def call(T=fake, ldt=100, G=fake, ldg=80, flags=0, work=null, wb=0, b=16):
        return lib.randutv_factor_lower(100, 80, b, 1, T, ldt, G, ldg, null, 100, null, 80, 0,
                                        0.0, 0, flags, work, wb, None, null)
    assert call(b=0) == -2
    assert call(T=null) == -4
    assert call(ldg=79) == -5        # G has n = 80 rows
    assert call(flags=1) == -6
    assert call(flags=2) == -7
    assert call() == -12
    assert call(work=vp(4096), wb=16) == -901
