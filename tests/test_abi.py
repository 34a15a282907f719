"""Host-only checks of the C ABI: the library loads, exports every declared
symbol and validates descriptors without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfch.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pfch_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2204_07247_amd import pfch
    L = pfch.lib()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(pfch.EXPORTED)


def test_version_and_strerror():
    from paper_2204_07247_amd import pfch
    assert pfch.lib().pfch_version() == 1
    assert "max_iter" in pfch.strerror(pfch.PFCH_E_NOCONV)
    assert pfch.strerror(12345) == "unknown error"


def test_struct_sizes_match_header_layout():
    from paper_2204_07247_amd import pfch
    # 3 + 5 + 3 + 8 doubles, then 6 + 3 + 1 int32
    assert ctypes.sizeof(pfch.InstanceDesc) == 19 * 8 + 10 * 4
    # dnorm, beta[4], mass, rnorm, gain; iters, fft_pairs, status, guess
    assert ctypes.sizeof(pfch.Stats) == 8 * 8 + 4 * 4
    assert pfch.Stats.rnorm_inf.offset == 6 * 8
    assert pfch.Stats.gain.offset == 7 * 8


def _desc(**kw):
    from paper_2204_07247_amd import pfch
    base = dict(model="pfc", scheme="mp", shape=(64, 64), lengths=(64.0, 64.0), eps=0.25)
    base.update(kw)
    return pfch.make_desc(**base)


@pytest.mark.parametrize("kw,code", [
    (dict(), 0),
    (dict(model="fch", eps=0.1, eta1=0.145, eta2=0.2), 0),
    (dict(shape=(2048, 8), lengths=(1.0, 1.0)), 0),
    (dict(shape=(64, 100)), -7),
    (dict(shape=(4096, 64)), -7),
    (dict(shape=(8, 8, 8), lengths=(1.0, 1.0, 1.0)), 0),            # 3D PFC
    (dict(shape=(8, 24, 8), lengths=(1.0, 1.0, 1.0)), -7),          # y length not supported
    (dict(model="fch", shape=(8, 8, 8), lengths=(1.0, 1.0, 1.0), eps=0.1), -7),  # 3D FCH
    (dict(shape=(64, 192), lengths=(64.0, 192.0)), 0),              # mixed radix 2D
    (dict(shape=(64, 96), lengths=(64.0, 96.0)), -7),
    (dict(s=0.0), -1),
    (dict(tol=-1.0), -1),
    (dict(max_iter=0), -1),
    (dict(etas=()), 0),                       # no momentum: Alg. 1
    (dict(scheme="lbdf2"), 0),
    (dict(scheme=4), -1),
    (dict(lengths=(0.0, 1.0)), -1),
    (dict(model="fch", eps=0.0), -1),
    (dict(mobility=float("nan")), -1),
])
def test_descriptor_validation(kw, code):
    from paper_2204_07247_amd import pfch
    assert pfch.validate_desc(_desc(**kw)) == code


def test_invalid_model_and_reserved_fields():
    from paper_2204_07247_amd import pfch
    d = _desc()
    d.model = 7
    assert pfch.validate_desc(d) == pfch.PFCH_E_INVAL
    d = _desc()
    d.reserved = 1
    assert pfch.validate_desc(d) == pfch.PFCH_E_INVAL
    d = _desc()
    d.guess = 1
    assert pfch.validate_desc(d) == pfch.PFCH_OK
    d.guess = 2
    assert pfch.validate_desc(d) == pfch.PFCH_E_INVAL


def test_fno_sizes_and_argument_checks_on_host():
    """Parameter count equals the reference network's; invalid network
    shapes and arguments are rejected before any device work."""
    from oracle import fno as ofno
    from paper_2204_07247_amd import pfch
    for w, m, l in ((32, 16, 4), (4, 3, 2), (8, 5, 3)):
        assert pfch.fno_num_params(w, m, l) == ofno.n_params(w, m, l)
    assert pfch.fno_num_params(0, 3, 2) == pfch.PFCH_E_INVAL
    assert pfch.fno_num_params(65, 3, 2) == pfch.PFCH_E_INVAL
    L = pfch.lib()
    h = ctypes.c_void_p()
    # 2M > Ny, 2M > Nx, zero batch, null output
    assert L.pfch_fno_create(4, 7, 2, 12, 12, 1, None, ctypes.byref(h)) == pfch.PFCH_E_INVAL
    assert L.pfch_fno_create(4, 3, 2, 12, 4, 1, None, ctypes.byref(h)) == pfch.PFCH_E_INVAL
    assert L.pfch_fno_create(4, 3, 2, 12, 12, 0, None, ctypes.byref(h)) == pfch.PFCH_E_INVAL
    assert L.pfch_fno_create(4, 3, 2, 12, 12, 1, None, None) == pfch.PFCH_E_INVAL
    for w, m, l in ((16, 8, 4), (3, 2, 2)):
        assert pfch.fno_num_params(w, m, l, ndim=3) == ofno.n_params(w, m, l, ndim=3)
    # 3D: 2M > Nz, null output
    assert L.pfch_fno_create_3d(4, 3, 2, 4, 12, 12, 1, None, ctypes.byref(h)) == pfch.PFCH_E_INVAL
    assert L.pfch_fno_create_3d(4, 3, 2, 12, 12, 12, 1, None, None) == pfch.PFCH_E_INVAL
    assert L.pfch_fno_forward(None, None, None, 1) == pfch.PFCH_E_INVAL
    assert L.pfch_fno_adam_step(None, 1e-3, 0.9, 0.999, 1e-8, 1) == pfch.PFCH_E_INVAL
    assert L.pfch_set_fno(None, 0, None, None) == pfch.PFCH_E_INVAL


def test_create_rejects_bad_arguments_before_device_work():
    from paper_2204_07247_amd import pfch
    L = pfch.lib()
    h = ctypes.c_void_p()
    d = _desc(s=-1.0)
    assert L.pfch_create(ctypes.byref(d), 1, None, ctypes.byref(h)) == pfch.PFCH_E_INVAL
    assert L.pfch_create(ctypes.byref(_desc()), 0, None, ctypes.byref(h)) == pfch.PFCH_E_INVAL
    assert L.pfch_step(None, None, None) == pfch.PFCH_E_INVAL
    assert L.pfch_set_stats_detail(None, 1) == pfch.PFCH_E_INVAL
    assert L.pfch_set_stats_detail(None, 2) == pfch.PFCH_E_INVAL
    assert L.pfch_time_kernels(None, 0.1, 1, None) == pfch.PFCH_E_INVAL
    ad = pfch.AdaptDesc(1e-4, 1e-3, 1.0, pfch.EST_AUTO, 0)
    res = (pfch.AdaptResult * 1)()
    assert L.pfch_step_adaptive(None, ctypes.byref(ad), res) == pfch.PFCH_E_INVAL
    assert L.pfch_rhs(None, 0, None, None) == pfch.PFCH_E_INVAL


@pytest.mark.parametrize("compiler,std", [("gcc", "-std=c99"), ("g++", "-std=c++11")])
def test_header_compiles_as_c_and_cxx(tmp_path, compiler, std):
    """The public header is plain C (usable without HIP or C++ headers)."""
    import shutil
    import subprocess
    cc = shutil.which(compiler)
    if cc is None:
        pytest.skip(f"{compiler} not available")
    src = tmp_path / ("h.c" if compiler == "gcc" else "h.cpp")
    src.write_text('#include "pfch.h"\n'
                   "int main(void) {\n"
                   "  pfch_instance_desc d;\n"
                   "  pfch_stats s;\n"
                   "  (void)d; (void)s;\n"
                   "  return pfch_version() > 0 ? 0 : 1;\n"
                   "}\n")
    r = subprocess.run([cc, std, "-Wall", "-Wextra", "-Werror", "-pedantic", "-fsyntax-only",
                        "-I", os.path.dirname(HEADER), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def _bits(x):
    import struct
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def test_stop_record_decision_on_the_host():
    """The host's reading of a solve's stop record (Alg. 2's stopping rule):
    a record still marked running is never reported as a result, with zero
    iterations or otherwise; a stop at j means j + 1 iterations; the cap,
    a non-finite norm and the preconditioner flag map to their errors."""
    from paper_2204_07247_amd import pfch
    tol_hit = _bits(7.5e-11)
    # running record (stop_iter -1, norm 0): internal error, not OK
    rc, it, dn = pfch.stop_status(-1, 0, 0, 1000)
    assert rc == pfch.PFCH_E_INTERNAL and it == 0
    rc, it, dn = pfch.stop_status(-1, 0, tol_hit, 1000)
    assert rc == pfch.PFCH_E_INTERNAL
    # stopped at j = 11: twelve iterations, the norm reported
    rc, it, dn = pfch.stop_status(11, 0, tol_hit, 1000)
    assert (rc, it, dn) == (pfch.PFCH_OK, 12, 7.5e-11)
    rc, it, dn = pfch.stop_status(0, 0, tol_hit, 1000)
    assert (rc, it) == (pfch.PFCH_OK, 1)
    # the cap
    rc, it, dn = pfch.stop_status(1000, 0, _bits(3e-6), 1000)
    assert (rc, it) == (pfch.PFCH_E_NOCONV, 1000)
    # non-finite norms
    for bad in (float("inf"), float("nan")):
        rc, it, dn = pfch.stop_status(4, 0, _bits(bad), 1000)
        assert (rc, it) == (pfch.PFCH_E_NONFINITE, 5)
    # preconditioner flag wins, also on a record that never started
    rc, it, dn = pfch.stop_status(-1, 1, 0, 1000)
    assert (rc, it) == (pfch.PFCH_E_PRECOND, 0)
    # argument checks
    L = pfch.lib()
    i = ctypes.c_int32()
    d = ctypes.c_double()
    assert L.pfch_stop_status(0, 0, 0, 0, ctypes.byref(i), ctypes.byref(d)) == pfch.PFCH_E_INVAL
    assert L.pfch_stop_status(0, 0, 0, 10, None, ctypes.byref(d)) == pfch.PFCH_E_INVAL
    assert "internal" in pfch.strerror(pfch.PFCH_E_INTERNAL)
