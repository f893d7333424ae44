"""Thin ctypes binding of include/aderdg.h, include/aderdg2d.h,
include/aderdg3d.h, include/aderdg_lim.h and include/aderdg_lim2d.h (argument
marshalling only).

Every entry point keeps its C name.  Buffers may be torch tensors on the HIP
device (their data_ptr() is passed) or raw integer device addresses.  All
compute happens in libaderdg.so; if the library is missing, load() raises.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.environ.get("ADERDG_LIB", os.path.join(HERE, "libaderdg.so"))

ADERDG_OK = 0
ADERDG_E_INVAL = -1
ADERDG_E_NOMEM = -2
ADERDG_E_DEVICE = -3
ADERDG_E_NOCONV = -4
ADERDG_E_NONPHYS = -5

PDE_ADVECTION, PDE_EULER, PDE_EULER_REACT, PDE_SWE = 0, 1, 2, 3
FP64, FP32_PREDICTOR = 0, 1
BC_PERIODIC = 0
CFL_SUBCELL, CFL_NODAL = 0, 1
SCHEME_DG, SCHEME_FV = 0, 1
INNER_PICARD, INNER_NEWTON = 0, 1
NVARS = {PDE_ADVECTION: 1, PDE_EULER: 3, PDE_EULER_REACT: 5, PDE_SWE: 3}

EXPORTS = ["aderdg_init", "aderdg_predict", "aderdg_correct", "aderdg_step", "aderweno_step",
           "aderdg_free", "aderdg_set_stream", "aderdg_sweep_count", "aderdg_contraction_count",
           "aderdg_operators", "aderdg_conserved_totals", "aderdg_step_noalloc", "aderdg_user_init",
           "aderdg_user_compile_check", "aderdg_set_waves", "aderdg_autotune", "aderdg_last_error"]
EXPORTS_2D = ["aderdg2d_init", "aderdg2d_predict", "aderdg2d_step", "aderdg2d_sweep_count",
              "aderdg2d_free"]
EXPORTS_3D = ["aderdg3d_init", "aderdg3d_predict", "aderdg3d_step", "aderdg3d_sweep_count",
              "aderdg3d_free"]
EXPORTS_LIM = ["aderdg_lim_init", "aderdg_lim_project", "aderdg_lim_step", "aderdg_lim_counters",
               "aderdg_lim_free"]
LIM_PERIODIC, LIM_TRANSMISSIVE = 0, 1
EXPORTS_LIM2D = ["aderdg2d_lim_init", "aderdg2d_lim_project", "aderdg2d_lim_step", "aderdg2d_lim_counters",
                 "aderdg2d_lim_free"]


class PdeDesc(ctypes.Structure):
    _fields_ = [("pde", ctypes.c_int32), ("nvars", ctypes.c_int32), ("gamma", ctypes.c_double),
                ("g", ctypes.c_double), ("omega", ctypes.c_double), ("adv_speed", ctypes.c_double)]


class Config(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("bc", ctypes.c_int32), ("ncells", ctypes.c_int64),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("cfl", ctypes.c_double),
                ("fixed_dt", ctypes.c_double), ("cfl_mode", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("picard_tol", ctypes.c_double),
                ("picard_max_iter", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("inner", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Config2D(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("cells_x", ctypes.c_int64), ("cells_y", ctypes.c_int64),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double),
                ("y0", ctypes.c_double), ("y1", ctypes.c_double),
                ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("fixed_dt", ctypes.c_double),
                ("picard_tol", ctypes.c_double), ("picard_max_iter", ctypes.c_int32),
                ("scheme", ctypes.c_int32)]


class Config3D(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("cells_x", ctypes.c_int64), ("cells_y", ctypes.c_int64), ("cells_z", ctypes.c_int64),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double),
                ("y1", ctypes.c_double), ("z0", ctypes.c_double), ("z1", ctypes.c_double),
                ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("fixed_dt", ctypes.c_double),
                ("picard_tol", ctypes.c_double), ("picard_max_iter", ctypes.c_int32),
                ("scheme", ctypes.c_int32)]


class LimConfig(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("bc", ctypes.c_int32), ("ncells", ctypes.c_int64),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("gamma", ctypes.c_double),
                ("cfl", ctypes.c_double), ("dims", ctypes.c_int32), ("picard_max_iter", ctypes.c_int32),
                ("picard_tol", ctypes.c_double), ("weno_degree", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Lim2DConfig(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("bc", ctypes.c_int32), ("cells_x", ctypes.c_int64),
                ("cells_y", ctypes.c_int64), ("x0", ctypes.c_double), ("x1", ctypes.c_double),
                ("y0", ctypes.c_double), ("y1", ctypes.c_double), ("cfl", ctypes.c_double),
                ("gamma", ctypes.c_double), ("picard_tol", ctypes.c_double),
                ("picard_max_iter", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class AderdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"aderdg error {code}: {msg}")
        self.code = code


_lib = None


def load(path=None):
    """Load libaderdg.so (once).  Raises if it is absent: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIBPATH
    if not os.path.exists(p):
        raise FileNotFoundError(f"{p} not built; run `python -m paper_2409_12483_amd.build`")
    # PyTorch provides the device memory and streams the library works on;
    # load it (and the HIP runtime it brings) before the library, so that one
    # runtime serves both
    import torch  # noqa: F401
    lib = ctypes.CDLL(p)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.aderdg_init.argtypes = [ctypes.POINTER(PdeDesc), ctypes.POINTER(Config), i32, vp, ctypes.POINTER(vp)]
    lib.aderdg_predict.argtypes = [vp, i32, vp, dbl, dbl, vp, vp]
    lib.aderdg_correct.argtypes = [vp, i32, vp, vp, dbl, dbl, vp]
    lib.aderdg_step.argtypes = [vp, ctypes.POINTER(vp), vp, vp, vp, vp, i32]
    lib.aderweno_step.argtypes = [vp, ctypes.POINTER(vp), vp, vp, vp, vp, i32]
    lib.aderdg_free.argtypes = [vp]
    lib.aderdg_set_stream.argtypes = [vp, vp]
    lib.aderdg_sweep_count.argtypes = [vp, i32, ctypes.POINTER(i64)]
    lib.aderdg_contraction_count.argtypes = [vp, i32, ctypes.POINTER(i64)]
    lib.aderdg_operators.argtypes = [i32, ctypes.POINTER(dbl), i64]
    lib.aderdg_conserved_totals.argtypes = [vp, i32, vp, vp]
    lib.aderdg_user_init.argtypes = [ctypes.c_char_p, i32, ctypes.POINTER(dbl), ctypes.POINTER(Config), vp,
                                     ctypes.POINTER(vp)]
    lib.aderdg_user_compile_check.argtypes = [ctypes.c_char_p, i32, i32, i32, ctypes.c_char_p, i64]
    lib.aderdg_step_noalloc.argtypes = [ctypes.POINTER(PdeDesc), ctypes.POINTER(Config), vp, vp, vp,
                                        vp, vp, i32, vp]
    lib.aderdg_set_waves.argtypes = [vp, i32]
    lib.aderdg_autotune.argtypes = [vp, vp, i32, vp]
    lib.aderdg_last_error.argtypes = []
    lib.aderdg_last_error.restype = ctypes.c_char_p
    lib.aderdg2d_init.argtypes = [ctypes.POINTER(Config2D), vp, ctypes.POINTER(vp)]
    lib.aderdg2d_predict.argtypes = [vp, vp, dbl, dbl, vp, vp]
    lib.aderdg2d_step.argtypes = [vp, vp, vp, vp, vp, vp, i32]
    lib.aderdg2d_sweep_count.argtypes = [vp, ctypes.POINTER(i64)]
    lib.aderdg2d_free.argtypes = [vp]
    lib.aderdg3d_init.argtypes = [ctypes.POINTER(Config3D), vp, ctypes.POINTER(vp)]
    lib.aderdg3d_predict.argtypes = [vp, vp, dbl, dbl, vp, vp]
    lib.aderdg3d_step.argtypes = [vp, vp, vp, vp, vp, vp, i32]
    lib.aderdg3d_sweep_count.argtypes = [vp, ctypes.POINTER(i64)]
    lib.aderdg3d_free.argtypes = [vp]
    lib.aderdg_lim_init.argtypes = [ctypes.POINTER(LimConfig), vp, ctypes.POINTER(vp)]
    lib.aderdg_lim_project.argtypes = [vp, vp, vp]
    lib.aderdg_lim_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, i32]
    lib.aderdg_lim_counters.argtypes = [vp, ctypes.POINTER(i64)]
    lib.aderdg_lim_free.argtypes = [vp]
    lib.aderdg2d_lim_init.argtypes = [ctypes.POINTER(Lim2DConfig), vp, ctypes.POINTER(vp)]
    lib.aderdg2d_lim_project.argtypes = [vp, vp, vp]
    lib.aderdg2d_lim_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, i32]
    lib.aderdg2d_lim_counters.argtypes = [vp, ctypes.POINTER(i64)]
    lib.aderdg2d_lim_free.argtypes = [vp]
    for name in EXPORTS[:-1] + EXPORTS_2D + EXPORTS_3D + EXPORTS_LIM + EXPORTS_LIM2D:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _check(rc):
    if rc != ADERDG_OK:
        raise AderdgError(rc, aderdg_last_error())
    return rc


def _current_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def pde_desc(pde, gamma=1.4, g=9.81, omega=1.0, adv_speed=1.0):
    return PdeDesc(pde, NVARS[pde], gamma, g, omega, adv_speed)


def config(N, ncells, x0=0.0, x1=1.0, cfl=0.4, fixed_dt=0.0, cfl_mode=CFL_SUBCELL,
           precision=FP64, picard_tol=0.0, picard_max_iter=0, scheme=SCHEME_DG, inner=INNER_PICARD):
    return Config(N, BC_PERIODIC, ncells, x0, x1, cfl, fixed_dt, cfl_mode, precision,
                  picard_tol, picard_max_iter, scheme, inner, 0)


def aderdg_init(pdes, cfgs, stream=None):
    """Returns an opaque handle (int).  stream: HIP stream handle (default: torch's current)."""
    lib = load()
    n = len(pdes)
    P = (PdeDesc * n)(*pdes)
    C = (Config * n)(*cfgs)
    h = ctypes.c_void_p()
    s = _current_stream() if stream is None else stream
    _check(lib.aderdg_init(P, C, n, s, ctypes.byref(h)))
    return h.value


def aderdg_predict(h, k, u, t, dt, q_out, iters_out=None):
    return _check(load().aderdg_predict(h, k, _ptr(u), t, dt, _ptr(q_out), _ptr(iters_out)))


def aderdg_correct(h, k, u, q, t, dt, u_next):
    return _check(load().aderdg_correct(h, k, _ptr(u), _ptr(q), t, dt, _ptr(u_next)))


def _ptr_array(states):
    arr = (ctypes.c_void_p * len(states))(*[_ptr(s) for s in states])
    return arr


def aderdg_step(h, u, t, t_end, dt, status, nsteps):
    return _check(load().aderdg_step(h, _ptr_array(u), _ptr(t), _ptr(t_end), _ptr(dt), _ptr(status), nsteps))


def aderweno_step(h, v, t, t_end, dt, status, nsteps):
    return _check(load().aderweno_step(h, _ptr_array(v), _ptr(t), _ptr(t_end), _ptr(dt), _ptr(status), nsteps))


def aderdg_set_waves(h, waves):
    return _check(load().aderdg_set_waves(h, waves))


def aderdg_autotune(h, u, steps, nprob=None):
    """Returns the workgroup size now used by each problem's group (list of ints)."""
    n = nprob if nprob is not None else len(u)
    out = (ctypes.c_int32 * n)()
    _check(load().aderdg_autotune(h, _ptr_array(u), steps, out))
    return list(out)


def aderdg_step_noalloc(pde, cfg, u, t, t_end, dt, status, nsteps, stream=None):
    """One problem, no handle, no device allocation (library-resident scratch).
    stream: HIP stream handle (default: torch's current)."""
    s = _current_stream() if stream is None else stream
    return _check(load().aderdg_step_noalloc(ctypes.byref(pde), ctypes.byref(cfg), _ptr(u), _ptr(t),
                                             _ptr(t_end), _ptr(dt), _ptr(status), nsteps, s))


def aderdg_free(h):
    return _check(load().aderdg_free(h))


def aderdg_set_stream(h, stream):
    return _check(load().aderdg_set_stream(h, stream))


def aderdg_sweep_count(h, k):
    v = ctypes.c_int64()
    _check(load().aderdg_sweep_count(h, k, ctypes.byref(v)))
    return v.value


def aderdg_contraction_count(h, k):
    v = ctypes.c_int64()
    _check(load().aderdg_contraction_count(h, k, ctypes.byref(v)))
    return v.value


def aderdg_user_init(model_source, nvars, cfg, params=(1.4, 9.81, 1.0, 1.0), stream=None):
    """Handle of one DG problem of a runtime-compiled user model (see include/aderdg.h)."""
    lib = load()
    h = ctypes.c_void_p()
    p = (ctypes.c_double * 4)(*params)
    s = _current_stream() if stream is None else stream
    _check(lib.aderdg_user_init(model_source.encode(), nvars, p, ctypes.byref(cfg), s, ctypes.byref(h)))
    return h.value


def aderdg_user_compile_check(model_source, nvars, N, precision=FP64):
    """(ok, compiler log) for a user model, compiled on the host only."""
    buf = ctypes.create_string_buffer(1 << 16)
    rc = load().aderdg_user_compile_check(model_source.encode(), nvars, N, precision, buf, len(buf))
    return rc == ADERDG_OK, buf.value.decode(errors="replace")


def aderdg_conserved_totals(h, k, u, out):
    """Enqueue the conserved totals of problem k's state u into the device array out [M]."""
    return _check(load().aderdg_conserved_totals(h, k, _ptr(u), _ptr(out)))


def aderdg_operators(N):
    """Host-only operator tables: dict of numpy arrays (no device involved)."""
    import numpy as np
    n = N + 1
    Ns = 2 * N + 1
    cap = 2 * n + 3 * n * n + 2 * n + 2 * Ns * n
    buf = (ctypes.c_double * cap)()
    got = load().aderdg_operators(N, buf, cap)
    if got < 0:
        _check(got)
    a = np.frombuffer(buf, dtype=np.float64, count=cap).copy()
    o = 0
    out = {}
    for name, size, shape in [("xi", n, (n,)), ("w", n, (n,)), ("ktil", n * n, (n, n)),
                              ("kappa", n * n, (n, n)), ("Dtil", n * n, (n, n)),
                              ("psi0", n, (n,)), ("psi1", n, (n,)), ("P", Ns * n, (Ns, n)),
                              ("R", n * Ns, (n, Ns))]:
        out[name] = a[o:o + size].reshape(shape)
        o += size
    return out


def aderdg_last_error():
    msg = load().aderdg_last_error()
    return msg.decode() if msg else ""


# ------------------------------------------------------------------ 2-D ----
def config2d(N, cells_x, cells_y, extent=(0.0, 1.0, 0.0, 1.0), gamma=1.4, cfl=0.4, fixed_dt=0.0,
             precision=FP64, picard_tol=0.0, picard_max_iter=0, scheme=SCHEME_DG):
    x0, x1, y0, y1 = extent
    return Config2D(N, precision, cells_x, cells_y, x0, x1, y0, y1, gamma, cfl, fixed_dt,
                    picard_tol, picard_max_iter, scheme)


def aderdg2d_init(cfg, stream=None):
    lib = load()
    h = ctypes.c_void_p()
    st = _current_stream() if stream is None else stream
    _check(lib.aderdg2d_init(ctypes.byref(cfg), st, ctypes.byref(h)))
    return h.value


def aderdg2d_predict(h, u, t, dt, q_out, iters_out=None):
    return _check(load().aderdg2d_predict(h, _ptr(u), t, dt, _ptr(q_out), _ptr(iters_out)))


def aderdg2d_step(h, u, t, t_end, dt, status, nsteps):
    return _check(load().aderdg2d_step(h, _ptr(u), _ptr(t), _ptr(t_end), _ptr(dt), _ptr(status), nsteps))


def aderdg2d_sweep_count(h):
    out = ctypes.c_int64()
    _check(load().aderdg2d_sweep_count(h, ctypes.byref(out)))
    return out.value


def aderdg2d_free(h):
    return _check(load().aderdg2d_free(h))


# ------------------------------------------------------------------ 3-D ----
def config3d(N, cells, extent=(1.0, 1.0, 1.0), gamma=1.4, cfl=0.4, fixed_dt=0.0, precision=FP64,
             picard_tol=0.0, picard_max_iter=0, scheme=SCHEME_DG):
    """cells: (cx, cy, cz); extent: (Lx, Ly, Lz) of the domain [0, Lx] x [0, Ly] x [0, Lz]."""
    cx, cy, cz = cells
    return Config3D(N, precision, cx, cy, cz, 0.0, extent[0], 0.0, extent[1], 0.0, extent[2],
                    gamma, cfl, fixed_dt, picard_tol, picard_max_iter, scheme)


def aderdg3d_init(cfg, stream=None):
    lib = load()
    h = ctypes.c_void_p()
    st = _current_stream() if stream is None else stream
    _check(lib.aderdg3d_init(ctypes.byref(cfg), st, ctypes.byref(h)))
    return h.value


def aderdg3d_predict(h, u, t, dt, q_out, iters_out=None):
    return _check(load().aderdg3d_predict(h, _ptr(u), t, dt, _ptr(q_out), _ptr(iters_out)))


def aderdg3d_step(h, u, t, t_end, dt, status, nsteps):
    return _check(load().aderdg3d_step(h, _ptr(u), _ptr(t), _ptr(t_end), _ptr(dt), _ptr(status), nsteps))


def aderdg3d_sweep_count(h):
    out = ctypes.c_int64()
    _check(load().aderdg3d_sweep_count(h, ctypes.byref(out)))
    return out.value


def aderdg3d_free(h):
    return _check(load().aderdg3d_free(h))


# ------------------------------------------------------------- limited 1-D ----
def lim_config(N, ncells, bc=LIM_TRANSMISSIVE, x0=0.0, x1=1.0, gamma=1.4, cfl=0.4, dims=1,
               picard_tol=0.0, picard_max_iter=0, weno_degree=1):
    return LimConfig(N, bc, ncells, x0, x1, gamma, cfl, dims, picard_max_iter, picard_tol, weno_degree, 0)


def aderdg_lim_init(cfg, stream=None):
    lib = load()
    h = ctypes.c_void_p()
    st = _current_stream() if stream is None else stream
    _check(lib.aderdg_lim_init(ctypes.byref(cfg), st, ctypes.byref(h)))
    return h.value


def aderdg_lim_project(h, u, v):
    return _check(load().aderdg_lim_project(h, _ptr(u), _ptr(v)))


def aderdg_lim_step(h, u, v, troubled, t, t_end, dt, status, nsteps):
    return _check(load().aderdg_lim_step(h, _ptr(u), _ptr(v), _ptr(troubled), _ptr(t), _ptr(t_end),
                                         _ptr(dt), _ptr(status), nsteps))


def aderdg_lim_counters(h):
    """(troubled cell-steps, first-order fallback steps, steps taken, predictor sweeps) since init."""
    out = (ctypes.c_int64 * 4)()
    _check(load().aderdg_lim_counters(h, out))
    return tuple(out)


def aderdg_lim_free(h):
    return _check(load().aderdg_lim_free(h))


# ------------------------------------------------------------- limited 2-D ----
def lim2d_config(N, cells_x, cells_y, bc=LIM_TRANSMISSIVE, extent=(-1.0, 1.0, -1.0, 1.0), gamma=1.4, cfl=0.4,
                 picard_tol=0.0, picard_max_iter=0):
    x0, x1, y0, y1 = extent
    return Lim2DConfig(N, bc, cells_x, cells_y, x0, x1, y0, y1, cfl, gamma, picard_tol, picard_max_iter, 0)


def aderdg2d_lim_init(cfg, stream=None):
    lib = load()
    h = ctypes.c_void_p()
    st = _current_stream() if stream is None else stream
    _check(lib.aderdg2d_lim_init(ctypes.byref(cfg), st, ctypes.byref(h)))
    return h.value


def aderdg2d_lim_project(h, u, v):
    return _check(load().aderdg2d_lim_project(h, _ptr(u), _ptr(v)))


def aderdg2d_lim_step(h, u, v, troubled, t, t_end, dt, status, nsteps):
    return _check(load().aderdg2d_lim_step(h, _ptr(u), _ptr(v), _ptr(troubled), _ptr(t), _ptr(t_end),
                                           _ptr(dt), _ptr(status), nsteps))


def aderdg2d_lim_counters(h):
    """(troubled cell-steps, first-order redo steps, 0, candidate predictor sweeps) since init."""
    out = (ctypes.c_int64 * 4)()
    _check(load().aderdg2d_lim_counters(h, out))
    return tuple(out)


def aderdg2d_lim_free(h):
    return _check(load().aderdg2d_lim_free(h))
