"""The C-ABI library loads without a GPU, exports every function that
include/lb.h declares, and rejects invalid parameters on the host."""
import ctypes
import os

import numpy as np
import pytest

from paper_0906_3611_amd import lb


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(lb.LIB_PATH):
        pytest.fail("liblbsoft.so is not built (run __graft_entry__.build())")
    return lb.load()


def test_every_declared_function_is_exported(L):
    names = lb.header_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(L, n), n
    assert L.lb_abi_version() == 4


def _params(**kw):
    p = lb.lb_params()
    p.nx, p.ny = kw.get("nx", 16), kw.get("ny", 16)
    p.boundary = kw.get("boundary", lb.LB_PERIODIC)
    p.precision = kw.get("precision", lb.LB_FP64)
    p.tau[0] = p.tau[1] = kw.get("tau", 1.0)
    p.rho0 = kw.get("rho0", 0.83)
    p.G_a[0] = p.G_a[1] = -9.0
    p.G_r[0] = p.G_r[1] = 8.1
    p.G_AB = 0.405
    p.u_wall = kw.get("u_wall", 0.0)
    return p


@pytest.mark.parametrize("bad", [dict(nx=4), dict(ny=3), dict(tau=0.5), dict(rho0=0.0),
                                 dict(boundary=7), dict(precision=3), dict(u_wall=float("nan")),
                                 dict(tau=float("inf"))])
def test_invalid_params_rejected(L, bad):
    p = _params(**bad)
    n = ctypes.c_size_t()
    assert L.lb_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == lb.LB_E_INVAL
    h = ctypes.c_void_p()
    assert L.lb_create(ctypes.byref(p), None, ctypes.byref(h)) == lb.LB_E_INVAL
    assert not h.value
    # the failed create leaves its reason for this thread (null handle)
    why = L.lb_last_error(None).decode()
    assert why and why != "null handle", why


@pytest.mark.parametrize("nx,precision", [(30_000_000, lb.LB_FP64), (60_000_000, lb.LB_FP32_DEV),
                                          (100_000_000, lb.LB_FP32_MOM), (200_000_000, lb.LB_FP32_DEV)])
def test_rows_beyond_32bit_offsets_rejected(L, nx, precision):
    """A row whose bytes reach 2^31 (the kernels' in-row offsets are 32-bit)
    is refused on the host, though it has fewer than 2^30 sites."""
    p = _params(nx=nx, ny=5, precision=precision)
    n = ctypes.c_size_t()
    assert L.lb_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == lb.LB_E_INVAL
    h = ctypes.c_void_p()
    assert L.lb_create(ctypes.byref(p), None, ctypes.byref(h)) == lb.LB_E_INVAL
    assert not h.value
    assert "32-bit" in L.lb_last_error(None).decode()


@pytest.mark.parametrize("nx,precision", [(14_000_000, lb.LB_FP64), (29_000_000, lb.LB_FP32_DEV),
                                          (89_000_000, lb.LB_FP32_MOM)])
def test_longest_rows_within_32bit_offsets_accepted(L, nx, precision):
    p = _params(nx=nx, ny=5, precision=precision)
    n = ctypes.c_size_t()
    assert L.lb_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == lb.LB_OK


def test_workspace_size_accounts_for_both_buffers(L):
    for prec, elem in ((lb.LB_FP64, 8), (lb.LB_FP32_DEV, 4)):
        p = _params(nx=100, ny=70, precision=prec)
        n = ctypes.c_size_t()
        assert L.lb_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == lb.LB_OK
        pitch = 128  # nx rounded up to 32 elements
        assert n.value >= 2 * 18 * pitch * 70 * elem


def test_status_strings(L):
    for code in (0, -1, -2, -3, -4, -5):
        assert L.lb_strerror(code)
    # a thread with no failed create reads "null handle" for a null handle
    import threading
    seen = []
    t = threading.Thread(target=lambda: seen.append(L.lb_last_error(None)))
    t.start()
    t.join()
    assert seen == [b"null handle"]
    assert L.lb_step(None, 1) == lb.LB_E_INVAL
    assert L.lb_current_step(None) == -1


@pytest.mark.parametrize("nx,ny,seed,phi", [(64, 48, 1, 0.7), (17, 9, 3, 0.5), (8, 8, 2, 0.9),
                                            (200, 60, 11, 1.0), (33, 5, 4, 0.0), (256, 192, 9, 0.6)])
def test_library_disc_fields_match_the_input_generator(L, nx, ny, seed, phi):
    """lb_disc_fields (host code of the library) reproduces the Python
    generator bit for bit: both draw the same counters and take the same
    minimum-image decisions in FP64."""
    from paper_0906_3611_amd import inputs
    ra, rb = inputs.disc_fields(nx, ny, seed, phi)
    ga, gb = lb.disc_fields(nx, ny, seed, phi)
    assert np.array_equal(ra, ga) and np.array_equal(rb, gb)


def test_library_disc_fields_reject_bad_specs(L):
    for kw in (dict(phi=1.5), dict(phi=-0.1), dict(phi=0.5, rmin=0.0), dict(phi=0.5, rmin=5.0, rmax=4.0)):
        phi = kw.pop("phi")
        with pytest.raises(lb.LBError):
            lb.disc_fields(16, 16, 1, phi, **kw)


def test_pool_schedule_names_checked_before_any_device_call():
    with pytest.raises(ValueError):
        lb.Pool(1 << 20, schedule="fifo")


def test_tune_cache_file_is_loaded_filtered_and_rewritten(L, tmp_path):
    """lb_set_tune_cache reads a results file (skipping lines that do not
    parse or hold out-of-range values) and writes the table back whole."""
    path = tmp_path / "tune.txt"
    path.write_text("abi4/gfx950/f32dev/periodic/launch/256x256 8 0 1 4 12.5\n"
                    "garbage line\n"
                    "abi4/gfx950/f64/walls/launch/70x45 16 7 0 1 30.0\n"   # prefetch out of range
                    "abi4/gfx950/f32dev/periodic/launch/64x64 8 0 1 3 12.5\n"  # tiles per group
                    "abi4/gfx950/f32mom/periodic/launch/128x128 4 0 0 1 9.0\n")
    assert L.lb_set_tune_cache(str(path).encode()) == lb.LB_OK
    lines = sorted(path.read_text().splitlines())
    assert lines == ["abi4/gfx950/f32dev/periodic/launch/256x256 8 0 1 4 12.5",
                     "abi4/gfx950/f32mom/periodic/launch/128x128 4 0 0 1 9"]
    # written under a temporary name of this process and renamed into place
    assert [p.name for p in tmp_path.iterdir()] == ["tune.txt"]
    assert L.lb_set_tune_cache(None) == lb.LB_OK
    assert L.lb_set_tune_cache(str(tmp_path / "missing_dir" / "t.txt").encode()) == lb.LB_E_INVAL
    assert L.lb_set_tune_cache(None) == lb.LB_OK


def test_probe_library_exports_its_header():
    """libhbmprobe.so (the copy-ceiling probe the benchmark runs) loads
    without a GPU and exports every function include/hbm_probe.h declares;
    invalid arguments are refused on the host before any launch."""
    import re
    from paper_0906_3611_amd import _build
    assert os.path.exists(_build.PROBE_LIB), "libhbmprobe.so is not built"
    P = ctypes.CDLL(_build.PROBE_LIB)
    hdr = os.path.join(os.path.dirname(lb.HEADER), "hbm_probe.h")
    txt = re.sub(r"/\*.*?\*/", "", open(hdr).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(hbm_[a-z_]+)\s*\(", txt)))
    assert names == ["hbm_copy"]
    for n in names:
        assert hasattr(P, n), n
    P.hbm_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                           ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    # null buffers, a size that is not a multiple of 16, a bad unroll: refused
    assert P.hbm_copy(None, None, 4096, 1, 256, 0, 1, None) == -1
    assert P.hbm_copy(16, 32, 100, 1, 256, 0, 1, None) == -1
    assert P.hbm_copy(16, 32, 4096, 1, 256, 0, 3, None) == -1


def test_kolmogorov_force_drives_the_requested_mode(L):
    """lb_kolmogorov_force (host only) returns the body-force amplitude for
    which the oracle's steady first mode of u_x (Sec. VIII, Eq. (66)) is the
    requested U0, within the lattice's O(k^2) error at tau = 1.3, ny = 64
    (0.5%), for both signs of U0; invalid arguments are refused."""
    import oracle
    for u0 in (0.01, -0.004):
        g = ctypes.c_double()
        assert L.lb_kolmogorov_force(u0, 64, 1.3, ctypes.byref(g)) == lb.LB_OK
        p = oracle.Params(nx=4, ny=64, tau=(1.3, 1.3), rho0=1.0, Ga=(0, 0), Gr=(0, 0), Gab=0.0,
                          g_body=g.value)
        f0 = oracle.init_equilibrium(p, np.full((64, 4), 0.6), np.full((64, 4), 0.4))
        f, _ = oracle.run(p, f0, 16000)
        assert oracle.totals(p, f)["u_mode"] == pytest.approx(u0, rel=5e-3)
    g = ctypes.c_double()
    for args in ((0.01, 4, 1.0), (0.01, 64, 0.5), (float("nan"), 64, 1.0), (0.01, 64, float("inf"))):
        assert L.lb_kolmogorov_force(*args, ctypes.byref(g)) == lb.LB_E_INVAL
    assert L.lb_kolmogorov_force(0.01, 64, 1.0, None) == lb.LB_E_INVAL


def test_null_handles_are_refused_on_the_host(L):
    """Every verb on a null handle returns LB_E_INVAL before any device
    call."""
    assert L.lb_step(None, 1) == lb.LB_E_INVAL
    assert L.lb_sync(None) == lb.LB_E_INVAL
    assert L.lb_batch_step(None, 1) == lb.LB_E_INVAL
    assert L.lb_pool_advance(None, 1) == lb.LB_E_INVAL
