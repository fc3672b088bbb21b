"""Python binding of the mclbm C ABI (include/mclbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
libmclbm.so.  The functions below carry the names of the C entry points; the
``Sim`` class wraps one simulation whose device arena is a torch tensor and
whose work goes to torch's current HIP stream.  Importing this module fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np
# torch first: it loads its own HIP runtime, and the library must bind to that
# one.  Loaded the other way round, the process holds two HIP runtimes and the
# library's finds no device.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmclbm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2502_00920_amd.build` "
                      "(hipcc, gfx950); there is no fallback implementation")

_lib = C.CDLL(LIB_PATH)

# ---- enums (include/mclbm.h) ---------------------------------------------------------
MCLBM_OK, MCLBM_EINVAL, MCLBM_ETOOSMALL, MCLBM_EHIP, MCLBM_EUNSTABLE, MCLBM_ESTATE = 0, -1, -2, -3, -4, -5
MATERIAL = {"svk": 0, "neohooke": 1, "linear": 2}
PRECISION = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
SIDE = {"left": 0, "right": 1, "bottom": 2, "top": 3}
BC = {"dirichlet": 0, "neumann": 1, "periodic": 2}
LOAD = {"zero": 0, "const": 1, "disp_ramp": 2, "linear_ramp": 3, "sin2_ramp": 4,
        "sin_pulse": 5, "gauss": 6, "ricker": 7, "table": 8}
FIELD = {"u": 0, "j": 1, "r": 2, "pi": 3, "h": 4, "p": 5, "s": 6}


class mclbm_params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("material", C.c_int32),
                ("precision", C.c_int32), ("dx", C.c_double), ("rho0", C.c_double),
                ("mu", C.c_double), ("nu", C.c_double), ("tau", C.c_double),
                ("body", C.c_double * 2), ("tau_plus", C.c_double),
                ("growth_limit", C.c_double), ("extrap", C.c_int32), ("corner", C.c_int32),
                ("boundary_order", C.c_int32), ("time_levels", C.c_int32), ("diag_every", C.c_int32),
                ("reserved_", C.c_int32)]


class mclbm_side_spec(C.Structure):
    _fields_ = [("bc", C.c_int32), ("kind", C.c_int32), ("amp", C.c_double * 2),
                ("t0", C.c_double), ("t1", C.c_double), ("width", C.c_double),
                ("table", C.POINTER(C.c_double)), ("table_len", C.c_int64)]


class mclbm_server_config(C.Structure):
    _fields_ = [("precision", C.c_int32), ("steps_per_round", C.c_int32), ("max_active", C.c_int32)]


class mclbm_diag_out(C.Structure):
    _fields_ = [("step", C.c_int64), ("momentum", C.c_double * 2), ("ekin", C.c_double),
                ("max_u", C.c_double), ("nonfinite", C.c_int32), ("growth", C.c_int32),
                ("cfl_excess", C.c_int32), ("pad_", C.c_int32), ("first_bad_step", C.c_int64)]


_vp, _i, _i64, _sz = C.c_void_p, C.c_int, C.c_int64, C.c_size_t
_sig = {
    "mclbm_plan": (_i, [C.POINTER(mclbm_params), C.POINTER(_sz), C.POINTER(_sz), C.POINTER(C.c_double)]),
    "mclbm_create": (_i, [C.POINTER(mclbm_params), _vp, _sz, _vp, C.POINTER(_vp)]),
    "mclbm_set_side": (_i, [_vp, _i, C.POINTER(mclbm_side_spec)]),
    "mclbm_init": (_i, [_vp, _vp, _vp, _i]),
    "mclbm_step": (_i, [_vp, _i64]),
    "mclbm_step_timed": (_i, [_vp, _i64, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "mclbm_step_checked": (_i, [_vp, _i64, _i64, C.POINTER(_i64)]),
    "mclbm_copy": (_i, [_vp, _vp, _sz, _vp]),
    "mclbm_stepno": (_i64, [_vp]),
    "mclbm_field_components": (_i, [_i]),
    "mclbm_read": (_i, [_vp, _i, _vp, _i]),
    "mclbm_diag": (_i, [_vp, C.POINTER(mclbm_diag_out)]),
    "mclbm_diag_noalloc": (_i, [_vp, C.POINTER(mclbm_diag_out)]),
    "mclbm_state_bytes": (_sz, [_vp]),
    "mclbm_save": (_i, [_vp, _vp, _sz, _i]),
    "mclbm_load": (_i, [_vp, _vp, _sz, _i]),
    "mclbm_destroy": (_i, [_vp]),
    "mclbm_last_error": (C.c_char_p, []),
    "mclbm_server_plan": (_i, [C.POINTER(mclbm_server_config), C.POINTER(_sz)]),
    "mclbm_server_create": (_i, [C.POINTER(mclbm_server_config), _vp, _sz, _vp, C.POINTER(_vp)]),
    "mclbm_server_submit": (_i, [_vp, C.POINTER(mclbm_params), C.POINTER(mclbm_side_spec), _vp, _i64, _vp,
                                 C.POINTER(_i64)]),
    "mclbm_server_progress": (_i, [_vp, C.POINTER(_i64), C.c_int32, C.POINTER(C.c_int32)]),
    "mclbm_server_result": (_i, [_vp, _i64, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "mclbm_server_steps": (_i, [_vp, _i64, C.POINTER(_i64)]),
    "mclbm_server_counts": (_i, [_vp, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i64)]),
    "mclbm_server_destroy": (_i, [_vp]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class MclbmError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: status {code}: {mclbm_last_error()}")


def _check(rc: int, where: str) -> None:
    if rc != MCLBM_OK:
        raise MclbmError(rc, where)


# ---- the C entry points, same names ------------------------------------------------------

def mclbm_last_error() -> str:
    return _lib.mclbm_last_error().decode()


def mclbm_plan(p: mclbm_params):
    """(arena_bytes, dt) for these parameters (the alignment: mclbm_plan_align)."""
    nbytes, align, dt = _sz(0), _sz(0), C.c_double(0)
    _check(_lib.mclbm_plan(C.byref(p), C.byref(nbytes), C.byref(align), C.byref(dt)), "mclbm_plan")
    return nbytes.value, dt.value


def mclbm_plan_align(p: mclbm_params) -> int:
    """The arena alignment mclbm_plan reports."""
    align = _sz(0)
    _check(_lib.mclbm_plan(C.byref(p), None, C.byref(align), None), "mclbm_plan")
    return align.value


def mclbm_create(p: mclbm_params, arena_ptr: int, arena_bytes: int, stream_ptr: int) -> int:
    h = _vp()
    _check(_lib.mclbm_create(C.byref(p), _vp(arena_ptr), arena_bytes, _vp(stream_ptr), C.byref(h)),
           "mclbm_create")
    return h.value


def mclbm_set_side(h: int, side: int, spec: mclbm_side_spec) -> None:
    _check(_lib.mclbm_set_side(_vp(h), side, C.byref(spec)), "mclbm_set_side")


def mclbm_init(h: int, u0_ptr: Optional[int], j0_ptr: Optional[int], on_device: int) -> None:
    _check(_lib.mclbm_init(_vp(h), _vp(u0_ptr), _vp(j0_ptr), on_device), "mclbm_init")


def mclbm_step(h: int, nsteps: int) -> None:
    _check(_lib.mclbm_step(_vp(h), int(nsteps)), "mclbm_step")


def mclbm_step_checked(h: int, nsteps: int, every: int):
    """(ok, steps run): nsteps in runs of `every`, stopped at the first run
    that leaves a displacement that is not finite or, with a growth limit, above it."""
    done = _i64(0)
    rc = _lib.mclbm_step_checked(_vp(h), int(nsteps), int(every), C.byref(done))
    if rc == MCLBM_EUNSTABLE:
        return False, done.value
    _check(rc, "mclbm_step_checked")
    return True, done.value


def mclbm_step_timed(h: int, nsteps: int):
    """(mean ms of one step, mean ms of its main kernel) over nsteps steps, from
    HIP events around each step's launches and after its main kernel."""
    ms, mm = C.c_double(0), C.c_double(0)
    _check(_lib.mclbm_step_timed(_vp(h), int(nsteps), C.byref(ms), C.byref(mm)), "mclbm_step_timed")
    return ms.value, mm.value


def mclbm_copy(dst_ptr: int, src_ptr: int, nbytes: int, stream_ptr: int) -> None:
    _check(_lib.mclbm_copy(_vp(dst_ptr), _vp(src_ptr), int(nbytes), _vp(stream_ptr)), "mclbm_copy")


def mclbm_stepno(h: int) -> int:
    return _lib.mclbm_stepno(_vp(h))


def mclbm_field_components(field: int) -> int:
    return _lib.mclbm_field_components(field)


def mclbm_read(h: int, field: int, dst_ptr: int, on_device: int) -> None:
    _check(_lib.mclbm_read(_vp(h), field, _vp(dst_ptr), on_device), "mclbm_read")


def mclbm_diag(h: int) -> mclbm_diag_out:
    out = mclbm_diag_out()
    rc = _lib.mclbm_diag(_vp(h), C.byref(out))
    if rc not in (MCLBM_OK, MCLBM_EUNSTABLE):
        _check(rc, "mclbm_diag")
    return out


def mclbm_diag_noalloc(h: int) -> mclbm_diag_out:
    """mclbm_diag with its scratch in the library's fixed device array."""
    out = mclbm_diag_out()
    rc = _lib.mclbm_diag_noalloc(_vp(h), C.byref(out))
    if rc not in (MCLBM_OK, MCLBM_EUNSTABLE):
        _check(rc, "mclbm_diag_noalloc")
    return out


def mclbm_state_bytes(h: int) -> int:
    return _lib.mclbm_state_bytes(_vp(h))


def mclbm_save(h: int, dst_ptr: int, nbytes: int, on_device: int) -> None:
    _check(_lib.mclbm_save(_vp(h), _vp(dst_ptr), int(nbytes), on_device), "mclbm_save")


def mclbm_load(h: int, src_ptr: int, nbytes: int, on_device: int) -> None:
    _check(_lib.mclbm_load(_vp(h), _vp(src_ptr), int(nbytes), on_device), "mclbm_load")


def mclbm_destroy(h: int) -> None:
    _lib.mclbm_destroy(_vp(h))


def mclbm_server_plan(cfg: mclbm_server_config) -> int:
    n = _sz(0)
    _check(_lib.mclbm_server_plan(C.byref(cfg), C.byref(n)), "mclbm_server_plan")
    return n.value


def mclbm_server_create(cfg: mclbm_server_config, pool_ptr: int, pool_bytes: int, stream_ptr: int) -> int:
    h = _vp()
    _check(_lib.mclbm_server_create(C.byref(cfg), _vp(pool_ptr), pool_bytes, _vp(stream_ptr), C.byref(h)),
           "mclbm_server_create")
    return h.value


def mclbm_server_submit(h: int, p: mclbm_params, sides, u0_ptr: Optional[int], nsteps: int,
                        u_out_ptr: int) -> int:
    arr = (mclbm_side_spec * 4)(*sides)
    rid = _i64(0)
    _check(_lib.mclbm_server_submit(_vp(h), C.byref(p), arr, _vp(u0_ptr), int(nsteps), _vp(u_out_ptr),
                                    C.byref(rid)), "mclbm_server_submit")
    return rid.value


def mclbm_server_progress(h: int, cap: int = 1024):
    ids = (_i64 * cap)()
    n = C.c_int32(0)
    _check(_lib.mclbm_server_progress(_vp(h), ids, cap, C.byref(n)), "mclbm_server_progress")
    return [ids[i] for i in range(n.value)]


def mclbm_server_result(h: int, rid: int):
    st, status = C.c_int32(0), C.c_int32(0)
    _check(_lib.mclbm_server_result(_vp(h), int(rid), C.byref(st), C.byref(status)), "mclbm_server_result")
    return st.value, status.value


def mclbm_server_counts(h: int):
    w, a, d = _i64(0), _i64(0), _i64(0)
    _check(_lib.mclbm_server_counts(_vp(h), C.byref(w), C.byref(a), C.byref(d)), "mclbm_server_counts")
    return w.value, a.value, d.value


def mclbm_server_steps(h: int, rid: int) -> int:
    n = _i64(0)
    _check(_lib.mclbm_server_steps(_vp(h), int(rid), C.byref(n)), "mclbm_server_steps")
    return n.value


def mclbm_server_destroy(h: int) -> None:
    _lib.mclbm_server_destroy(_vp(h))


# ---- convenience wrapper (torch owns the device memory and the stream) -------------------------

def make_params(nx, ny, *, mu, nu, tau, material="svk", precision="f64", rho0=1.0, dx=1.0,
                body=(0.0, 0.0), tau_plus=0.0, growth_limit=0.0, extrap=0, corner=0, boundary_order=1,
                time_levels=0, diag_every=0) -> mclbm_params:
    p = mclbm_params()
    p.nx, p.ny = int(nx), int(ny)
    p.material, p.precision = MATERIAL[material], PRECISION[precision]
    p.dx, p.rho0, p.mu, p.nu, p.tau = float(dx), float(rho0), float(mu), float(nu), float(tau)
    p.body[0], p.body[1] = float(body[0]), float(body[1])
    p.tau_plus = float(tau_plus or 0.0)
    p.growth_limit = float(growth_limit or 0.0)
    p.extrap = {"copy": 0, "linear": 1}.get(extrap, extrap)
    p.corner, p.boundary_order, p.diag_every = int(corner), int(boundary_order), int(diag_every)
    p.time_levels = {"text": 0, "listing": 1}.get(time_levels, time_levels)
    p.reserved_ = 0
    return p


def make_side(bc, kind="zero", amp=(0.0, 0.0), t0=0.0, t1=0.0, width=0.0, table=None) -> mclbm_side_spec:
    """A side spec; for kind "table", `table` is the program per step (the
    library copies it, but the array must live until the call that takes the
    spec returns: the spec keeps a reference in ``_keep``)."""
    s = mclbm_side_spec()
    s.bc, s.kind = BC[bc], LOAD[kind]
    s.amp[0], s.amp[1] = float(amp[0]), float(amp[1])
    s.t0, s.t1, s.width = float(t0), float(t1), float(width)
    if table is not None:
        t = np.ascontiguousarray(table, dtype=np.float64).reshape(-1)
        s.table = t.ctypes.data_as(C.POINTER(C.c_double))
        s.table_len = t.size
        s._keep = t
    return s


class Sim:
    """One simulation on a GPU.  Fields come back as float64 torch tensors
    [comp, ny, nx] on the device (or numpy arrays with ``host=True``)."""

    def __init__(self, nx, ny, *, mu, nu, tau, material="svk", precision="f64", rho0=1.0,
                 dx=1.0, body=(0.0, 0.0), tau_plus=0.0, growth_limit=0.0, extrap=0, corner=0,
                 boundary_order=1, time_levels=0, diag_every=0, device="cuda", stream=None):
        import torch
        self.torch = torch
        self.nx, self.ny = int(nx), int(ny)
        self.params = make_params(nx, ny, mu=mu, nu=nu, tau=tau, material=material,
                                  precision=precision, rho0=rho0, dx=dx, body=body, tau_plus=tau_plus,
                                  growth_limit=growth_limit, extrap=extrap, corner=corner,
                                  boundary_order=boundary_order, time_levels=time_levels,
                                  diag_every=diag_every)
        self.arena_bytes, self.dt = mclbm_plan(self.params)
        self.device = torch.device(device)
        self.arena = torch.empty(self.arena_bytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = mclbm_create(self.params, self.arena.data_ptr(), self.arena_bytes,
                               self.stream.cuda_stream)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            try:
                mclbm_destroy(h)
            except TypeError:  # interpreter shutdown: the module's globals are gone
                pass

    @property
    def handle(self) -> int:
        return self._h

    @property
    def n(self) -> int:
        return mclbm_stepno(self._h)

    def set_side(self, side, bc, kind="zero", amp=(0.0, 0.0), t0=0.0, t1=0.0, width=0.0, table=None):
        mclbm_set_side(self._h, SIDE[side], make_side(bc, kind, amp, t0, t1, width, table))

    def init(self, u0=None, j0=None):
        t = self.torch

        def dev(a):
            if a is None:
                return None
            return t.as_tensor(np.asarray(a, dtype=np.float64)).reshape(2, self.ny, self.nx) \
                .to(self.device).contiguous()

        u, j = dev(u0), dev(j0)
        mclbm_init(self._h, None if u is None else u.data_ptr(), None if j is None else j.data_ptr(), 1)
        self._keep = (u, j)  # alive until the copies on the stream have run
        self.stream.synchronize()
        self._keep = None

    def step(self, n: int = 1):
        mclbm_step(self._h, n)

    def step_checked(self, n: int, every: int = 100):
        """Advance n steps, checking the displacement every `every` steps; returns
        (ok, steps run), ok False when a check found a value that is not finite
        or a |u| above the growth limit."""
        return mclbm_step_checked(self._h, n, every)

    def step_timed(self, n: int):
        """Advance n steps; returns (mean ms of one step, mean ms of its main
        kernel, march_kernel of the fused step)."""
        return mclbm_step_timed(self._h, n)

    def read(self, field: str, host: bool = True):
        nc = mclbm_field_components(FIELD[field])
        out = self.torch.empty((nc, self.ny, self.nx), dtype=self.torch.float64, device=self.device)
        mclbm_read(self._h, FIELD[field], out.data_ptr(), 1)
        return out.cpu().numpy() if host else out

    def diag(self) -> Dict:
        d = mclbm_diag(self._h)
        return {"step": d.step, "momentum": np.array([d.momentum[0], d.momentum[1]]),
                "ekin": d.ekin, "max_u": d.max_u, "nonfinite": bool(d.nonfinite),
                "growth": bool(d.growth), "cfl_excess": bool(d.cfl_excess),
                "first_bad_step": int(d.first_bad_step)}

    def save(self, host: bool = False):
        """A checkpoint (header and state) in a device tensor, or with host=True
        in a numpy byte array."""
        n = mclbm_state_bytes(self._h)
        if host:
            buf = np.empty(n, dtype=np.uint8)
            mclbm_save(self._h, buf.ctypes.data, n, 0)
            return buf
        buf = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        mclbm_save(self._h, buf.data_ptr(), n, 1)
        return buf

    def load(self, buf):
        """Continue from a checkpoint of save() (device tensor or numpy array)."""
        if isinstance(buf, np.ndarray):
            b = np.ascontiguousarray(buf, dtype=np.uint8)
            mclbm_load(self._h, b.ctypes.data, b.nbytes, 0)
        else:
            mclbm_load(self._h, buf.data_ptr(), buf.numel() * buf.element_size(), 1)


def sim_from_workload(w, precision="f64", **kw) -> Sim:
    """A Sim set up with the sides of a workloads.Workload (not yet initialised)."""
    s = Sim(w.nx, w.ny, mu=w.mu, nu=w.nu, tau=w.tau, material=w.material, precision=precision,
            rho0=w.rho0, dx=w.dx, **kw)
    for side, sd in w.sides.items():
        s.set_side(side, sd.bc, sd.kind, sd.amp, sd.t0, sd.t1, sd.width)
    return s


class Server:
    """A continuous-batching server over a torch-allocated device pool and a
    stream of its own (graph capture needs one).  ``submit`` queues a request
    and returns its id; ``progress`` runs one scheduling turn and returns the
    ids it finished; ``result(id)`` gives (state, status, u) with u the final
    displacement [2, ny, nx] as a numpy array once done."""

    def __init__(self, precision="f32", steps_per_round=32, max_active=64, pool_bytes=8 << 30,
                 device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.cfg = mclbm_server_config(PRECISION[precision], int(steps_per_round), int(max_active))
        self.precision = precision
        self.reserved = mclbm_server_plan(self.cfg)
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(device=self.device)
        self._h = mclbm_server_create(self.cfg, self.pool.data_ptr(), int(pool_bytes), self.stream.cuda_stream)
        self._out: Dict[int, np.ndarray] = {}
        self._keep: Dict[int, object] = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            try:
                mclbm_server_destroy(h)
            except TypeError:  # interpreter shutdown
                pass

    def submit(self, nx, ny, *, mu, nu, tau, material, sides, nsteps, u0=None, rho0=1.0, dx=1.0,
               body=(0.0, 0.0), tau_plus=0.0, growth_limit=0.0, extrap=0, corner=0) -> int:
        """sides: {"left": (bc, kind, amp, t0, t1, width[, table]) or bc, ...}; missing sides are free."""
        p = make_params(nx, ny, mu=mu, nu=nu, tau=tau, material=material, precision=self.precision,
                        rho0=rho0, dx=dx, body=body, tau_plus=tau_plus, growth_limit=growth_limit,
                        extrap=extrap, corner=corner)
        specs = []
        for name in ("left", "right", "bottom", "top"):
            spec = sides.get(name, "neumann")
            args = (spec,) if isinstance(spec, str) else tuple(spec)
            specs.append(make_side(*args))
        out = np.empty((2, int(ny), int(nx)), dtype=np.float64)
        u0a = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64).reshape(2, ny, nx)
        rid = mclbm_server_submit(self._h, p, specs, None if u0a is None else u0a.ctypes.data, nsteps,
                                  out.ctypes.data)
        self._out[rid] = out
        return rid

    def progress(self):
        return mclbm_server_progress(self._h)

    def result(self, rid):
        state, status = mclbm_server_result(self._h, rid)
        return state, status, (self._out.get(rid) if state == 2 else None)

    def counts(self):
        return mclbm_server_counts(self._h)

    def steps(self, rid) -> int:
        """Steps the request has run (fewer than asked when it was stopped as unstable)."""
        return mclbm_server_steps(self._h, rid)

    def drain(self):
        """Run turns until every submitted request is done; returns the finished ids in order."""
        done = []
        while True:
            done += self.progress()
            w, a, _ = self.counts()
            if w == 0 and a == 0:
                return done
