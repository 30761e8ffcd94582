"""Python binding of liblbsoft (include/lb.h): argument marshalling only.

Every step of the lattice Boltzmann update runs in the library's HIP
kernels.  PyTorch supplies the device workspace (a uint8 CUDA tensor) and
the HIP stream (torch's current stream), so library work interleaves with
torch work and torch's events can time it.  If the compiled library is
missing, load() raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbsoft.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lb.h")

LB_OK, LB_E_INVAL, LB_E_NOMEM, LB_E_DEVICE, LB_E_UNSTABLE, LB_E_STATE = 0, -1, -2, -3, -4, -5
LB_PERIODIC, LB_COUETTE_Y = 0, 1
LB_FP64, LB_FP32_DEV, LB_FP32_MOM = 0, 1, 2


class LBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class lb_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("boundary", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("tau", ctypes.c_double * 2), ("rho0", ctypes.c_double),
                ("G_a", ctypes.c_double * 2), ("G_r", ctypes.c_double * 2), ("G_AB", ctypes.c_double),
                ("u_wall", ctypes.c_double), ("body_force", ctypes.c_double),
                ("body_force_x", ctypes.c_double), ("rho_ref", ctypes.c_double * 2),
                ("device_buffer", ctypes.c_void_p), ("device_bytes", ctypes.c_size_t)]


class lb_obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("mass", ctypes.c_double * 2), ("mom", ctypes.c_double * 2),
                ("mom_phys", ctypes.c_double * 2), ("pxy_kin", ctypes.c_double),
                ("wall_stress", ctypes.c_double * 2), ("avg_count", ctypes.c_int64),
                ("flags", ctypes.c_int32), ("pad_", ctypes.c_int32), ("u_mode", ctypes.c_double),
                ("i_ab", ctypes.c_double), ("phi_overlap", ctypes.c_double),
                ("phi_ref_sq", ctypes.c_double), ("ref_step", ctypes.c_int64)]


class lb_launch_info(ctypes.Structure):
    _fields_ = [("nstrips", ctypes.c_int32), ("nsegs", ctypes.c_int32), ("ntiles", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("pitch", ctypes.c_int32), ("workspace_bytes", ctypes.c_size_t),
                ("population_bytes", ctypes.c_size_t), ("seg_h", ctypes.c_int32),
                ("prefetch", ctypes.c_int32), ("stream_stores", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("tiles_per_group", ctypes.c_int32)]


_lib = None


def load():
    """Load liblbsoft.so (built by __graft_entry__.build()).  Raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: the HIP library has not been built "
                          "(run __graft_entry__.build())")
    # torch ships its own HIP runtime.  Loaded first, it is the one the
    # library binds to; loaded after the library, a second runtime would sit
    # in the process, to which torch's device memory and streams (the
    # workspace and stream handed to lb_create) mean nothing.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, dp, i64, i32 = ctypes.c_void_p, P(ctypes.c_double), ctypes.c_int64, ctypes.c_int32
    h = ctypes.c_void_p
    fd = ctypes.c_double
    sig = {
        "lb_abi_version": ([], ctypes.c_int),
        "lb_kolmogorov_force": ([fd, i32, fd, dp], ctypes.c_int),
        "lb_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "lb_last_error": ([h], ctypes.c_char_p),
        "lb_workspace_bytes": ([P(lb_params), P(ctypes.c_size_t)], ctypes.c_int),
        "lb_create": ([P(lb_params), vp, P(h)], ctypes.c_int),
        "lb_init": ([h, dp, dp, dp, dp], ctypes.c_int),
        "lb_init_noise": ([h, ctypes.c_uint64, ctypes.c_double, ctypes.c_double, ctypes.c_double],
                          ctypes.c_int),
        "lb_init_discs": ([h, ctypes.c_uint64] + [fd] * 7, ctypes.c_int),
        "lb_disc_fields": ([i32, i32, ctypes.c_uint64] + [fd] * 7 + [dp, dp], ctypes.c_int),
        "lb_step": ([h, i64], ctypes.c_int),
        "lb_observables": ([h, P(lb_obs)], ctypes.c_int),
        "lb_get_fields": ([h, dp, dp, dp, dp], ctypes.c_int),
        "lb_get_fields_noalloc": ([h, dp, dp, dp, dp], ctypes.c_int),
        "lb_get_populations": ([h, dp], ctypes.c_int),
        "lb_set_populations": ([h, dp, i64], ctypes.c_int),
        "lb_reset_averages": ([h], ctypes.c_int),
        "lb_set_overlap_reference": ([h], ctypes.c_int),
        "lb_batch_set_overlap_reference": ([h], ctypes.c_int),
        "lb_sync": ([h], ctypes.c_int),
        "lb_current_step": ([h], i64),
        "lb_get_launch_info": ([h, P(lb_launch_info)], ctypes.c_int),
        "lb_set_launch": ([h, i32, i32, i32, i32, i32], ctypes.c_int),
        "lb_destroy": ([h], None),
        "lb_batch_workspace_bytes": ([P(lb_params), i32, P(ctypes.c_size_t)], ctypes.c_int),
        "lb_batch_create": ([P(lb_params), i32, vp, ctypes.c_size_t, vp, P(h)], ctypes.c_int),
        "lb_batch_size": ([h], i32),
        "lb_batch_init": ([h, i32, dp, dp, dp, dp], ctypes.c_int),
        "lb_batch_init_noise": ([h, i32, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double], ctypes.c_int),
        "lb_batch_init_discs": ([h, i32, ctypes.c_uint64] + [fd] * 7, ctypes.c_int),
        "lb_batch_step": ([h, i64], ctypes.c_int),
        "lb_batch_observables": ([h, P(lb_obs)], ctypes.c_int),
        "lb_batch_get_fields": ([h, i32, dp, dp, dp, dp], ctypes.c_int),
        "lb_batch_get_populations": ([h, i32, dp], ctypes.c_int),
        "lb_batch_sync": ([h], ctypes.c_int),
        "lb_batch_reset_averages": ([h], ctypes.c_int),
        "lb_batch_get_launch_info": ([h, P(lb_launch_info)], ctypes.c_int),
        "lb_batch_set_launch": ([h, i32, i32, i32, i32, i32], ctypes.c_int),
        "lb_batch_autotune": ([h, i32, P(lb_launch_info), dp], ctypes.c_int),
        "lb_autotune": ([h, i32, P(lb_launch_info), dp], ctypes.c_int),
        "lb_set_tune_cache": ([ctypes.c_char_p], ctypes.c_int),
        "lb_batch_destroy": ([h], None),
        "lb_batch_last_error": ([h], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def header_functions() -> list[str]:
    """Names of the functions include/lb.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_]+)\s*\(", txt)))


def _dptr(a):
    if a is None:
        return ctypes.cast(None, ctypes.POINTER(ctypes.c_double))
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


DISC_DEFAULTS = dict(rmin=6.0, rmax=12.0, in_a=1.2, in_b=0.05, out_a=0.05, out_b=1.2)


def _disc_args(phi, kw):
    a = dict(DISC_DEFAULTS)
    unknown = set(kw) - set(a)
    if unknown:
        raise TypeError(f"unknown disc arguments {sorted(unknown)}")
    a.update(kw)
    return [float(phi)] + [float(a[k]) for k in ("rmin", "rmax", "in_a", "in_b", "out_a", "out_b")]


def disc_fields(nx, ny, seed, phi, **kw):
    """Host disc-emulsion densities of the library (lb_disc_fields):
    (rho_a, rho_b), each (ny, nx) float64."""
    L = load()
    ra = np.empty((ny, nx), np.float64)
    rb = np.empty((ny, nx), np.float64)
    rc = L.lb_disc_fields(int(nx), int(ny), int(seed), *_disc_args(phi, kw), _dptr(ra), _dptr(rb))
    if rc != 0:
        raise LBError(rc, "lb_disc_fields: " + L.lb_strerror(rc).decode())
    return ra, rb


def make_params(nx, ny, *, tau=(1.0, 1.0), rho0=0.83, G_a=(-9.0, -9.0), G_r=(8.1, 8.1),
                G_AB=0.405, boundary="periodic", u_wall=0.0, precision="fp64",
                rho_ref=(0.0, 0.0), body_force=0.0, body_force_x=0.0) -> lb_params:
    """An lb_params record (parameters of Sec. II, Eqs. (1), (2), (5))."""
    p = lb_params()
    p.nx, p.ny = int(nx), int(ny)
    p.boundary = {"periodic": LB_PERIODIC, "couette": LB_COUETTE_Y}[boundary]
    p.precision = {"fp64": LB_FP64, "fp32dev": LB_FP32_DEV, "fp32mom": LB_FP32_MOM}[precision]
    p.tau[0], p.tau[1] = tau
    p.rho0 = rho0
    p.G_a[0], p.G_a[1] = G_a
    p.G_r[0], p.G_r[1] = G_r
    p.G_AB = G_AB
    p.u_wall = u_wall
    p.body_force = body_force
    p.body_force_x = body_force_x
    p.rho_ref[0], p.rho_ref[1] = rho_ref
    return p


def set_tune_cache(path):
    """Persist autotuner results in a text file (lb_set_tune_cache); None stops."""
    L = load()
    rc = L.lb_set_tune_cache(None if path is None else os.fsencode(path))
    if rc != 0:
        raise LBError(rc, f"lb_set_tune_cache: cannot write {path}")


def kolmogorov_force(U0, ny, tau=1.0):
    """Body-force amplitude g that drives U_x = U0 sin(2 pi y / ny) (Sec. VIII),
    from the library (lb_kolmogorov_force)."""
    L = load()
    g = ctypes.c_double()
    rc = L.lb_kolmogorov_force(float(U0), int(ny), float(tau), ctypes.byref(g))
    if rc != 0:
        raise LBError(rc, "lb_kolmogorov_force: " + L.lb_strerror(rc).decode())
    return g.value


def _obs_dict(o) -> dict:
    return {"step": o.step, "mass": np.array(o.mass[:]), "mom": np.array(o.mom[:]),
            "mom_phys": np.array(o.mom_phys[:]), "pxy_kin": o.pxy_kin,
            "wall_stress": np.array(o.wall_stress[:]), "avg_count": o.avg_count,
            "flags": o.flags, "u_mode": o.u_mode, "i_ab": o.i_ab, "phi_overlap": o.phi_overlap,
            "phi_ref_sq": o.phi_ref_sq, "ref_step": o.ref_step}


def _info_dict(li) -> dict:
    return {k: getattr(li, k) for k, _ in lb_launch_info._fields_}


def _torch_workspace(nbytes):
    import torch
    buf = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
    return buf, torch.cuda.current_stream()


class _Handle:
    _destroy = ""
    _last_error = ""

    def _check(self, rc, what):
        if rc != LB_OK:
            h = getattr(self, "_h", None)
            # a null handle reads the reason of this thread's failed create
            msg = (getattr(self._lib, self._last_error)(h if h and h.value else None)
                   or b"").decode()
            raise LBError(rc, f"{what}: {self._lib.lb_strerror(rc).decode()}: {msg}")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            getattr(self._lib, self._destroy)(self._h)
            self._h = ctypes.c_void_p()
        self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Lattice(_Handle):
    """One two-species lattice on the current GPU.

    precision: "fp64" or "fp32dev"; boundary: "periodic" or "couette".
    With use_torch (default) the device workspace is a torch uint8 tensor and
    work runs on torch's current stream; otherwise the library allocates and
    uses the null stream.
    """
    _destroy = "lb_destroy"
    _last_error = "lb_last_error"

    def __init__(self, nx: int, ny: int, *, tau=(1.0, 1.0), rho0=0.83, G_a=(-9.0, -9.0),
                 G_r=(8.1, 8.1), G_AB=0.405, boundary="periodic", u_wall=0.0, precision="fp64",
                 rho_ref=(0.0, 0.0), body_force=0.0, body_force_x=0.0, use_torch=True,
                 stream=None):
        self._lib = load()
        self._h = ctypes.c_void_p()
        self.nx, self.ny = int(nx), int(ny)
        p = make_params(nx, ny, tau=tau, rho0=rho0, G_a=G_a, G_r=G_r, G_AB=G_AB, boundary=boundary,
                        u_wall=u_wall, precision=precision, rho_ref=rho_ref, body_force=body_force,
                        body_force_x=body_force_x)
        self.precision, self.boundary = precision, boundary
        nbytes = ctypes.c_size_t()
        self._check(self._lib.lb_workspace_bytes(ctypes.byref(p), ctypes.byref(nbytes)), "workspace")
        self._buf = None
        if use_torch:
            self._buf, cur = _torch_workspace(nbytes.value)
            p.device_buffer = self._buf.data_ptr()
            p.device_bytes = int(nbytes.value)
            self.stream = cur if stream is None else stream
            sptr = self.stream.cuda_stream
        else:
            self.stream = stream
            sptr = None if stream is None else int(stream)
        self._check(self._lib.lb_create(ctypes.byref(p), sptr, ctypes.byref(self._h)), "lb_create")
        self.params = p

    def init(self, rho_a, rho_b, ux=None, uy=None):
        shp = (self.ny, self.nx)
        ra, rb = _f64(rho_a, shp), _f64(rho_b, shp)
        vx = None if ux is None else _f64(ux, shp)
        vy = None if uy is None else _f64(uy, shp)
        self._check(self._lib.lb_init(self._h, _dptr(ra), _dptr(rb), _dptr(vx), _dptr(vy)), "lb_init")

    def init_noise(self, seed, mean_a, mean_b, amp):
        self._check(self._lib.lb_init_noise(self._h, int(seed), float(mean_a), float(mean_b),
                                            float(amp)), "lb_init_noise")

    def init_discs(self, seed, phi, **kw):
        """Disc emulsion (lb_init_discs); keyword defaults in DISC_DEFAULTS."""
        self._check(self._lib.lb_init_discs(self._h, int(seed), *_disc_args(phi, kw)),
                    "lb_init_discs")

    def step(self, n=1):
        self._check(self._lib.lb_step(self._h, int(n)), "lb_step")

    @property
    def t(self) -> int:
        return int(self._lib.lb_current_step(self._h))

    def observables(self) -> dict:
        o = lb_obs()
        self._check(self._lib.lb_observables(self._h, ctypes.byref(o)), "lb_observables")
        return _obs_dict(o)

    def fields(self) -> dict:
        ny, nx = self.ny, self.nx
        ra, rb = np.empty((ny, nx)), np.empty((ny, nx))
        u, up = np.empty((2, ny, nx)), np.empty((2, ny, nx))
        self._check(self._lib.lb_get_fields(self._h, _dptr(ra), _dptr(rb), _dptr(u), _dptr(up)),
                    "lb_get_fields")
        return {"rho": np.stack([ra, rb]), "u": u, "uphys": up}

    def populations(self) -> np.ndarray:
        f = np.empty((2, 9, self.ny, self.nx))
        self._check(self._lib.lb_get_populations(self._h, _dptr(f)), "lb_get_populations")
        return f

    def set_populations(self, f, step=0):
        f = _f64(f, (2, 9, self.ny, self.nx))
        self._check(self._lib.lb_set_populations(self._h, _dptr(f), int(step)), "lb_set_populations")

    def reset_averages(self):
        self._check(self._lib.lb_reset_averages(self._h), "lb_reset_averages")

    def set_overlap_reference(self):
        """Store phi = rho_A - rho_B now as the reference of the overlap sums."""
        self._check(self._lib.lb_set_overlap_reference(self._h), "lb_set_overlap_reference")

    def sync(self):
        self._check(self._lib.lb_sync(self._h), "lb_sync")

    def launch_info(self) -> dict:
        li = lb_launch_info()
        self._check(self._lib.lb_get_launch_info(self._h, ctypes.byref(li)), "lb_get_launch_info")
        return _info_dict(li)

    def set_launch(self, seg_h=-1, prefetch=-1, stream_stores=-1, use_graph=-1,
                   tiles_per_group=-1):
        """Tuning knobs (lb_set_launch); -1 keeps the current choice."""
        self._check(self._lib.lb_set_launch(self._h, int(seg_h), int(prefetch), int(stream_stores),
                                            int(use_graph), int(tiles_per_group)), "lb_set_launch")

    def autotune(self, steps=20) -> dict:
        """lb_autotune: keep the fastest launch shape; returns it with its
        time per step (us_per_step).  The state is unchanged."""
        li, us = lb_launch_info(), ctypes.c_double()
        self._check(self._lib.lb_autotune(self._h, int(steps), ctypes.byref(li), ctypes.byref(us)),
                    "lb_autotune")
        return dict(_info_dict(li), us_per_step=us.value)


class Batch(_Handle):
    """Independent lattices advanced by one kernel launch per step.

    specs: a list of keyword dicts for make_params (each with nx and ny), all
    of one precision and boundary type."""
    _destroy = "lb_batch_destroy"
    _last_error = "lb_batch_last_error"

    def __init__(self, specs, use_torch=True, stream=None):
        self._lib = load()
        self._h = ctypes.c_void_p()
        n = len(specs)
        arr = (lb_params * n)()
        self.shapes = []
        for i, sp in enumerate(specs):
            sp = dict(sp)
            nx, ny = sp.pop("nx"), sp.pop("ny")
            arr[i] = make_params(nx, ny, **sp)
            self.shapes.append((int(ny), int(nx)))
        self.n = n
        nbytes = ctypes.c_size_t()
        self._check(self._lib.lb_batch_workspace_bytes(arr, n, ctypes.byref(nbytes)), "workspace")
        self._buf = None
        if use_torch:
            self._buf, cur = _torch_workspace(nbytes.value)
            self.stream = cur if stream is None else stream
            bptr, sptr = self._buf.data_ptr(), self.stream.cuda_stream
        else:
            self.stream, bptr, sptr = stream, None, (None if stream is None else int(stream))
        self._check(self._lib.lb_batch_create(arr, n, bptr, int(nbytes.value), sptr,
                                              ctypes.byref(self._h)), "lb_batch_create")

    def init(self, i, rho_a, rho_b, ux=None, uy=None):
        shp = self.shapes[i]
        ra, rb = _f64(rho_a, shp), _f64(rho_b, shp)
        vx = None if ux is None else _f64(ux, shp)
        vy = None if uy is None else _f64(uy, shp)
        self._check(self._lib.lb_batch_init(self._h, int(i), _dptr(ra), _dptr(rb), _dptr(vx),
                                            _dptr(vy)), "lb_batch_init")

    def init_noise(self, i, seed, mean_a, mean_b, amp):
        self._check(self._lib.lb_batch_init_noise(self._h, int(i), int(seed), float(mean_a),
                                                  float(mean_b), float(amp)), "lb_batch_init_noise")

    def init_discs(self, i, seed, phi, **kw):
        self._check(self._lib.lb_batch_init_discs(self._h, int(i), int(seed), *_disc_args(phi, kw)),
                    "lb_batch_init_discs")

    def step(self, n=1):
        self._check(self._lib.lb_batch_step(self._h, int(n)), "lb_batch_step")

    def observables(self) -> list:
        arr = (lb_obs * self.n)()
        self._check(self._lib.lb_batch_observables(self._h, arr), "lb_batch_observables")
        return [_obs_dict(o) for o in arr]

    def fields(self, i) -> dict:
        ny, nx = self.shapes[i]
        ra, rb = np.empty((ny, nx)), np.empty((ny, nx))
        u, up = np.empty((2, ny, nx)), np.empty((2, ny, nx))
        self._check(self._lib.lb_batch_get_fields(self._h, int(i), _dptr(ra), _dptr(rb), _dptr(u),
                                                  _dptr(up)), "lb_batch_get_fields")
        return {"rho": np.stack([ra, rb]), "u": u, "uphys": up}

    def populations(self, i) -> np.ndarray:
        ny, nx = self.shapes[i]
        f = np.empty((2, 9, ny, nx))
        self._check(self._lib.lb_batch_get_populations(self._h, int(i), _dptr(f)),
                    "lb_batch_get_populations")
        return f

    def sync(self):
        self._check(self._lib.lb_batch_sync(self._h), "lb_batch_sync")

    def reset_averages(self):
        self._check(self._lib.lb_batch_reset_averages(self._h), "lb_batch_reset_averages")

    def set_overlap_reference(self):
        """As Lattice.set_overlap_reference, for every lattice of the batch."""
        self._check(self._lib.lb_batch_set_overlap_reference(self._h),
                    "lb_batch_set_overlap_reference")

    def launch_info(self) -> dict:
        li = lb_launch_info()
        self._check(self._lib.lb_batch_get_launch_info(self._h, ctypes.byref(li)),
                    "lb_batch_get_launch_info")
        return _info_dict(li)

    def set_launch(self, seg_h=-1, prefetch=-1, stream_stores=-1, use_graph=-1,
                   tiles_per_group=-1):
        """Tuning knobs (lb_batch_set_launch); seg_h applies to every lattice."""
        self._check(self._lib.lb_batch_set_launch(self._h, int(seg_h), int(prefetch),
                                                  int(stream_stores), int(use_graph),
                                                  int(tiles_per_group)),
                    "lb_batch_set_launch")

    def autotune(self, steps=20) -> dict:
        """lb_batch_autotune: keep the fastest launch shape; returns it with
        its time per step (us_per_step)."""
        li, us = lb_launch_info(), ctypes.c_double()
        self._check(self._lib.lb_batch_autotune(self._h, int(steps), ctypes.byref(li),
                                                ctypes.byref(us)), "lb_batch_autotune")
        return dict(_info_dict(li), us_per_step=us.value)


LB_JOB_QUEUED, LB_JOB_RUNNING, LB_JOB_DONE, LB_JOB_FAILED = 0, 1, 2, 3


class lb_pool_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("running", ctypes.c_int64), ("done", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("resident_bytes", ctypes.c_size_t), ("budget_bytes", ctypes.c_size_t),
                ("site_updates", ctypes.c_int64), ("ticks", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("clock", ctypes.c_double)]


def _load_pool_symbols(L):
    P = ctypes.POINTER
    h, dp, i64, i32 = ctypes.c_void_p, P(ctypes.c_double), ctypes.c_int64, ctypes.c_int32
    sig = {
        "lb_pool_create": ([ctypes.c_size_t, h, P(h)], ctypes.c_int),
        "lb_pool_destroy": ([h], None),
        "lb_pool_last_error": ([h], ctypes.c_char_p),
        "lb_pool_set_options": ([h, i32, i32], ctypes.c_int),
        "lb_pool_set_schedule": ([h, i32, i64, i64], ctypes.c_int),
        "lb_pool_job_bytes": ([P(lb_params)], ctypes.c_size_t),
        "lb_pool_submit_noise": ([h, P(lb_params), ctypes.c_uint64, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, i64, P(i64)], ctypes.c_int),
        "lb_pool_submit": ([h, P(lb_params), dp, dp, i64, P(i64)], ctypes.c_int),
        "lb_pool_advance": ([h, i64], ctypes.c_int),
        "lb_pool_job_state": ([h, i64, P(i32)], ctypes.c_int),
        "lb_pool_job_progress": ([h, i64, P(i64)], ctypes.c_int),
        "lb_pool_job_result": ([h, i64, P(lb_obs), dp, dp, dp], ctypes.c_int),
        "lb_pool_release": ([h, i64], ctypes.c_int),
        "lb_pool_get_stats": ([h, P(lb_pool_stats)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res


def job_bytes(**spec) -> int:
    """Device footprint of one pool job with these parameters."""
    L = load()
    _load_pool_symbols(L)
    sp = dict(spec)
    nx, ny = sp.pop("nx"), sp.pop("ny")
    return int(L.lb_pool_job_bytes(ctypes.byref(make_params(nx, ny, **sp))))


class Pool(_Handle):
    """Serving pool: jobs admitted under an HBM budget, advanced in launches
    per class, retired with their results copied to the host (see
    include/lb.h).  schedule: "srpt" (least remaining work advances, up to
    fill_sites sites; a job held back max_hold pool steps goes first) or
    "lockstep" (every resident job, every step)."""
    _destroy = "lb_pool_destroy"
    _last_error = "lb_pool_last_error"

    def __init__(self, budget_bytes, stream=None, keep_fields=True, use_graph=False,
                 schedule="srpt", fill_sites=0, max_hold=0):
        policies = {"lockstep": 0, "srpt": 1}
        if schedule not in policies:
            raise ValueError(f"schedule must be one of {sorted(policies)}, not {schedule!r}")
        self._lib = load()
        _load_pool_symbols(self._lib)
        self._h = ctypes.c_void_p()
        self._buf = None
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.shapes = {}
        self._check(self._lib.lb_pool_create(int(budget_bytes), stream.cuda_stream,
                                             ctypes.byref(self._h)), "lb_pool_create")
        self._check(self._lib.lb_pool_set_options(self._h, int(keep_fields), int(use_graph)),
                    "lb_pool_set_options")
        self._check(self._lib.lb_pool_set_schedule(self._h, policies[schedule], int(fill_sites),
                                                   int(max_hold)),
                    "lb_pool_set_schedule")

    def submit_noise(self, steps, seed, mean_a, mean_b, amp, **spec) -> int:
        sp = dict(spec)
        nx, ny = sp.pop("nx"), sp.pop("ny")
        p = make_params(nx, ny, **sp)
        jid = ctypes.c_int64()
        self._check(self._lib.lb_pool_submit_noise(self._h, ctypes.byref(p), int(seed), float(mean_a),
                                                   float(mean_b), float(amp), int(steps),
                                                   ctypes.byref(jid)), "lb_pool_submit_noise")
        self.shapes[jid.value] = (int(ny), int(nx))
        return jid.value

    def submit(self, steps, rho_a, rho_b, **spec) -> int:
        sp = dict(spec)
        nx, ny = sp.pop("nx"), sp.pop("ny")
        p = make_params(nx, ny, **sp)
        ra, rb = _f64(rho_a, (ny, nx)), _f64(rho_b, (ny, nx))
        jid = ctypes.c_int64()
        self._check(self._lib.lb_pool_submit(self._h, ctypes.byref(p), _dptr(ra), _dptr(rb),
                                             int(steps), ctypes.byref(jid)), "lb_pool_submit")
        self.shapes[jid.value] = (int(ny), int(nx))
        return jid.value

    def advance(self, n):
        self._check(self._lib.lb_pool_advance(self._h, int(n)), "lb_pool_advance")

    def state(self, jid) -> int:
        s = ctypes.c_int32()
        self._check(self._lib.lb_pool_job_state(self._h, int(jid), ctypes.byref(s)), "lb_pool_job_state")
        return s.value

    def progress(self, jid) -> int:
        """Steps the job has run so far."""
        n = ctypes.c_int64()
        self._check(self._lib.lb_pool_job_progress(self._h, int(jid), ctypes.byref(n)),
                    "lb_pool_job_progress")
        return n.value

    def times(self, jid):
        t = np.zeros(3)
        self._lib.lb_pool_job_result(self._h, int(jid), None, _dptr(None), _dptr(None), _dptr(t))
        return t

    def result(self, jid, fields=True) -> dict:
        o = lb_obs()
        t = np.zeros(3)
        ny, nx = self.shapes[jid]
        ra = np.empty((ny, nx)) if fields else None
        rb = np.empty((ny, nx)) if fields else None
        self._check(self._lib.lb_pool_job_result(self._h, int(jid), ctypes.byref(o), _dptr(ra),
                                                 _dptr(rb), _dptr(t)), "lb_pool_job_result")
        out = {"obs": _obs_dict(o), "times": t}
        if fields:
            out["rho"] = np.stack([ra, rb])
        return out

    def release(self, jid):
        self._check(self._lib.lb_pool_release(self._h, int(jid)), "lb_pool_release")

    def stats(self) -> dict:
        s = lb_pool_stats()
        self._check(self._lib.lb_pool_get_stats(self._h, ctypes.byref(s)), "lb_pool_get_stats")
        return {k: getattr(s, k) for k, _ in lb_pool_stats._fields_}
