"""ctypes binding of liblbm.so (include/lbm.h): argument marshalling only.

Every step of the method runs in the HIP kernels of the library; PyTorch provides the
device memory (tensors) and the stream handle.  There is no CPU fallback: if the
shared library is missing, `load()` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_LIBRARY selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("LBM_LIBRARY") or os.path.join(_HERE, "liblbm.so")
_lib = None

LBM_OK, LBM_EINVAL, LBM_EUNSTABLE, LBM_EHIP, LBM_ESTATE, LBM_ENOROOT = 0, -1, -2, -3, -4, -5
FP64, FP32_SHIFTED = 0, 1
BASE_CS, BASE_PR = 0, 1
SHAPE_NONE, SHAPE_SMOOTH, SHAPE_MODSMOOTH, SHAPE_PENG = 0, 1, 2, 3
VARIANT_AUTO, VARIANT_MARCH, VARIANT_BLOCK, VARIANT_BLOCK2, VARIANT_AA = 0, 1, 2, 3, 4
BATCH_AUTO, BATCH_PERSISTENT, BATCH_GROUPED = 0, 1, 2


class LbmEos(C.Structure):
    _fields_ = [
        ("base", C.c_int), ("shape", C.c_int),
        ("a", C.c_double), ("b", C.c_double), ("R", C.c_double), ("omega", C.c_double),
        ("Tr", C.c_double), ("scale", C.c_double), ("alpha", C.c_double), ("k_vap", C.c_double),
        ("r_theta", C.c_double),
        ("Tc", C.c_double), ("T", C.c_double),
        ("rho_v", C.c_double), ("rho_l", C.c_double), ("p_sat", C.c_double),
        ("rho_max", C.c_double), ("p_max_base", C.c_double),
        ("rho_min", C.c_double), ("p_min_base", C.c_double),
        ("p_sat_new", C.c_double), ("dP_liq", C.c_double),
        ("slope_v", C.c_double), ("slope_l", C.c_double),
        ("p_max", C.c_double), ("p_min", C.c_double),
        ("a1sq", C.c_double), ("b1", C.c_double), ("a3sq", C.c_double), ("b3", C.c_double),
        ("rho_m", C.c_double), ("theta", C.c_double), ("eps", C.c_double),
    ]


class LbmParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("walls", C.c_int), ("prec", C.c_int),
        ("var_tau", C.c_int), ("reduce_every", C.c_int), ("band_rows", C.c_int), ("kernel_variant", C.c_int),
        ("rho_wall_lo", C.c_double), ("rho_wall_hi", C.c_double),
        ("G", C.c_double), ("sigma", C.c_double),
        ("tau", C.c_double * 9),
        ("tau_l", C.c_double), ("tau_v", C.c_double), ("rho_v_tau", C.c_double), ("rho_l_tau", C.c_double),
        ("rho_ref", C.c_double),
        ("eos", LbmEos),
        ("tile_rows", C.c_int),
    ]


class LbmFdParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("var_tau", C.c_int), ("walls", C.c_int),
        ("h", C.c_double), ("dt", C.c_double), ("G", C.c_double), ("eps", C.c_double),
        ("tau_e", C.c_double), ("tau_nu", C.c_double),
        ("tau_l", C.c_double), ("tau_v", C.c_double), ("rho_v_tau", C.c_double), ("rho_l_tau", C.c_double),
        ("eos", LbmEos),
    ]


class LbmError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = load().lbm_last_error().decode(errors="replace")
        super().__init__("%s failed: %s (%s)" % (where, load().lbm_strerror(code).decode(), msg))


# every symbol declared in include/lbm.h, with its ctypes signature
def _signatures():
    vp, d, i, sz = C.c_void_p, C.c_double, C.c_int, C.c_size_t
    dp = C.POINTER(C.c_double)
    return {
        "lbm_eos_build": ([C.POINTER(LbmEos), d, dp], i),
        "lbm_eos_pressure": ([C.POINTER(LbmEos), d], d),
        "lbm_eos_slope": ([C.POINTER(LbmEos), d], d),
        "lbm_layout": ([C.POINTER(LbmParams), C.POINTER(C.c_int), C.POINTER(sz), C.POINTER(sz)], i),
        "lbm_describe": ([C.POINTER(LbmParams), C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)], i),
        "lbm_init": ([C.POINTER(vp), C.POINTER(LbmParams), vp, vp, vp, sz, vp, vp, vp, vp], i),
        "lbm_init_static": ([C.POINTER(vp), C.POINTER(LbmParams), vp, vp, vp, vp, vp, vp], i),
        "lbm_tile_shape": ([vp, C.POINTER(C.c_int), C.POINTER(C.c_int)], i),
        "lbm_step": ([vp, C.c_int64, vp], i),
        "lbm_status_check": ([vp, vp], i),
        "lbm_macros": ([vp, vp, vp, vp, vp, vp, vp, vp, dp, vp], i),
        "lbm_populations": ([vp, vp, vp], i),
        "lbm_history": ([vp, dp, i, C.POINTER(C.c_int), vp], i),
        "lbm_state": ([vp, C.POINTER(C.c_int64), C.POINTER(C.c_int)], i),
        "lbm_save": ([vp, vp, vp], i),
        "lbm_load": ([vp, vp, C.c_int64, vp], i),
        "lbm_destroy": ([vp], None),
        "lbm_batch_layout": ([i, C.POINTER(LbmParams), C.POINTER(sz), C.POINTER(sz), C.POINTER(C.c_int64)], i),
        "lbm_init_batched": ([C.POINTER(vp), i, C.POINTER(LbmParams), vp, vp, vp, sz, vp, vp, vp, vp], i),
        "lbm_step_batched": ([vp, C.c_int64, vp], i),
        "lbm_set_batch_mode": ([vp, i], i),
        "lbm_macros_batched": ([vp, vp, vp, vp, vp], i),
        "lbm_status_batched": ([vp, C.POINTER(C.c_int), vp], i),
        "lbm_destroy_batched": ([vp], None),
        "lbm_adjoint_layout": ([C.POINTER(LbmParams), i, C.POINTER(sz), C.POINTER(sz)], i),
        "lbm_set_checkpointing": ([vp, vp, sz, i], i),
        "lbm_set_recording": ([vp, vp, sz, C.c_int64], i),
        "lbm_adjoint": ([vp, vp, vp, sz, vp, sz, dp, vp, vp], i),
        "lbm_adjoint_fields": ([vp, vp, vp, vp, vp, sz, vp, sz, dp, vp, vp], i),
        "lbm_eos_set_knots": ([C.POINTER(LbmEos), d, d, d, d], i),
        "lbm_fd_layout": ([C.POINTER(LbmFdParams), C.POINTER(sz)], i),
        "lbm_fd_init": ([C.POINTER(vp), C.POINTER(LbmFdParams), vp, sz, vp, vp, vp, vp], i),
        "lbm_fd_step": ([vp, C.c_int64, vp], i),
        "lbm_fd_fields": ([vp, vp, vp, vp, vp], i),
        "lbm_fd_status": ([vp, vp], i),
        "lbm_fd_destroy": ([vp], None),
        "lbm_strerror": ([i], C.c_char_p),
        "lbm_last_error": ([], C.c_char_p),
    }


def load():
    """Load the in-tree liblbm.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        # torch first: its bundled HIP runtime is the one the library must share
        import torch  # noqa: F401

        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbm.so not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        _assert_single_hip_runtime()
        for name, (args, res) in _signatures().items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _assert_single_hip_runtime():
    try:
        maps = open("/proc/self/maps").read()
    except OSError:
        return
    paths = {ln.split()[-1] for ln in maps.splitlines() if "libamdhip64" in ln}
    if len(paths) > 1:
        raise RuntimeError("two HIP runtimes loaded in one process: %s" % sorted(paths))


def _check(code: int, where: str):
    if code != LBM_OK:
        raise LbmError(code, where)


# ---------------------------------------------------------------------------- EOS
def make_eos(base=BASE_CS, shape=SHAPE_NONE, a=0.5, b=4.0, R=1.0, omega=0.344, Tr=0.7, scale=1.0,
             alpha=1.0, k_vap=1.0, r_theta=0.0) -> LbmEos:
    e = LbmEos()
    e.base, e.shape = base, shape
    e.a, e.b, e.R, e.omega, e.Tr = a, b, R, omega, Tr
    e.scale, e.alpha, e.k_vap, e.r_theta = scale, alpha, k_vap, r_theta
    return e


def eos_build(e: LbmEos, G: float = -1.0) -> tuple[LbmEos, float]:
    s = C.c_double(0.0)
    _check(load().lbm_eos_build(C.byref(e), G, C.byref(s)), "lbm_eos_build")
    return e, s.value


def eos_pressure(e: LbmEos, rho: float) -> float:
    return load().lbm_eos_pressure(C.byref(e), float(rho))


def eos_slope(e: LbmEos, rho: float) -> float:
    return load().lbm_eos_slope(C.byref(e), float(rho))


def eos_set_knots(e: LbmEos, rho_max: float, p_max: float, rho_min: float, p_min: float) -> LbmEos:
    """Copy of a built Smooth / Modified Smooth EOS with the four loop knots replaced."""
    out = LbmEos()
    C.memmove(C.byref(out), C.byref(e), C.sizeof(LbmEos))
    _check(load().lbm_eos_set_knots(C.byref(out), rho_max, p_max, rho_min, p_min), "lbm_eos_set_knots")
    return out


def adjoint_layout(P: LbmParams, K: int) -> tuple[int, int]:
    rec, adj = C.c_size_t(0), C.c_size_t(0)
    _check(load().lbm_adjoint_layout(C.byref(P), int(K), C.byref(rec), C.byref(adj)), "lbm_adjoint_layout")
    return rec.value, adj.value


GRAD_NAMES = ("rho_max", "p_max", "rho_min", "p_min", "G", "sigma")


def make_params(nx, ny, eos: LbmEos, G=-1.0, sigma=0.0, tau=None, prec=FP64, rho_ref=None, walls=False,
                rho_wall_lo=0.0, rho_wall_hi=0.0, var_tau=False, tau_l=1.0, tau_v=1.0, rho_v_tau=None,
                rho_l_tau=None, reduce_every=0, band_rows=0, kernel_variant=0, tile_rows=0) -> LbmParams:
    """tile_rows: two-step tile height (0: the library's choice, -1: timed by lbm_init, else that height)."""
    P = LbmParams()
    P.nx, P.ny, P.walls, P.prec, P.var_tau, P.reduce_every = nx, ny, int(walls), prec, int(var_tau), reduce_every
    P.band_rows = band_rows
    P.kernel_variant = kernel_variant
    P.rho_wall_lo, P.rho_wall_hi = rho_wall_lo, rho_wall_hi
    P.G, P.sigma = G, sigma
    t = [1.0] * 9 if tau is None else list(tau)
    for k in range(9):
        P.tau[k] = t[k]
    P.tau_l, P.tau_v = tau_l, tau_v
    P.rho_v_tau = eos.rho_v if rho_v_tau is None else rho_v_tau
    P.rho_l_tau = eos.rho_l if rho_l_tau is None else rho_l_tau
    P.rho_ref = (eos.rho_v if rho_ref is None else rho_ref) if prec == FP32_SHIFTED else 0.0
    P.eos = eos
    P.tile_rows = tile_rows
    return P


def layout(P: LbmParams) -> tuple[int, int, int]:
    ld, pb, wb = C.c_int(0), C.c_size_t(0), C.c_size_t(0)
    _check(load().lbm_layout(C.byref(P), C.byref(ld), C.byref(pb), C.byref(wb)), "lbm_layout")
    return ld.value, pb.value, wb.value


def describe(P: LbmParams) -> tuple[int, int, int]:
    """(kernel variant, rows per band/block, wavefronts) the library picks for P."""
    v, b, w = C.c_int(0), C.c_int(0), C.c_int(0)
    _check(load().lbm_describe(C.byref(P), C.byref(v), C.byref(b), C.byref(w)), "lbm_describe")
    return v.value, b.value, w.value


# ---------------------------------------------------------------------------- lattice
class Lattice:
    """A lattice whose populations live in two torch byte tensors on a HIP device (one for
    VARIANT_AA, which updates it in place)."""

    def __init__(self, P: LbmParams, rho0, ux0=None, uy0=None, device="cuda", stream=None,
                 static_workspace: bool = False):
        """static_workspace: lbm_init_static (the library's own workspace and context for this device,
        which the next such Lattice on the device takes over) instead of lbm_init."""
        import torch

        self.torch = torch
        self.P = P
        self.nx, self.ny = P.nx, P.ny
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ld, pop_bytes, ws_bytes = layout(P)
        self.pop_bytes = pop_bytes
        nbuf = 1 if P.kernel_variant == VARIANT_AA else 2
        self.f = [torch.empty(pop_bytes, dtype=torch.uint8, device=self.device) for _ in range(nbuf)]
        fb = self.f[1].data_ptr() if nbuf == 2 else None
        self.ws = None if static_workspace else torch.zeros(ws_bytes, dtype=torch.uint8, device=self.device)
        shp = (self.ny, self.nx)
        r = self._dev(rho0, shp)
        u = None if ux0 is None else self._dev(ux0, shp)
        v = None if uy0 is None else self._dev(uy0, shp)
        h = C.c_void_p(0)
        up, vp_ = (u.data_ptr() if u is not None else None), (v.data_ptr() if v is not None else None)
        if static_workspace:
            _check(load().lbm_init_static(C.byref(h), C.byref(P), self.f[0].data_ptr(), fb,
                                          r.data_ptr(), up, vp_, self._s()), "lbm_init_static")
        else:
            _check(load().lbm_init(C.byref(h), C.byref(P), self.f[0].data_ptr(), fb,
                                   self.ws.data_ptr(), ws_bytes, r.data_ptr(), up, vp_, self._s()), "lbm_init")
        self._keep = (r, u, v)
        self._h = h

    def _dev(self, a, shp):
        t = self.torch
        if isinstance(a, t.Tensor):
            x = a.to(device=self.device, dtype=t.float64).contiguous()
        else:
            x = t.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=self.device)
        assert tuple(x.shape) == shp, (tuple(x.shape), shp)
        return x

    def _s(self):
        return C.c_void_p(self.stream.cuda_stream)

    def close(self):
        if getattr(self, "_h", None):
            load().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        _check(load().lbm_step(self._h, int(n), self._s()), "lbm_step")

    def check(self):
        _check(load().lbm_status_check(self._h, self._s()), "lbm_status_check")

    def tile_shape(self) -> tuple[int, int]:
        """(output rows, wavefronts per workgroup) of the two-step tile this lattice runs."""
        r, w = C.c_int(0), C.c_int(0)
        _check(load().lbm_tile_shape(self._h, C.byref(r), C.byref(w)), "lbm_tile_shape")
        return r.value, w.value

    def macros(self) -> dict:
        t = self.torch
        shp = (self.ny, self.nx)
        out = {k: t.empty(shp, dtype=t.float64, device=self.device) for k in ("rho", "ux", "uy", "psi", "p", "Fx", "Fy")}
        mm = (C.c_double * 3)()
        _check(load().lbm_macros(self._h, *[out[k].data_ptr() for k in ("rho", "ux", "uy", "psi", "p", "Fx", "Fy")],
                                 mm, self._s()), "lbm_macros")
        out["mass_mom"] = (mm[0], mm[1], mm[2])
        return out

    def mass_momentum(self) -> tuple[float, float, float]:
        mm = (C.c_double * 3)()
        _check(load().lbm_macros(self._h, None, None, None, None, None, None, None, mm, self._s()), "lbm_macros")
        return mm[0], mm[1], mm[2]

    def populations(self):
        t = self.torch
        out = t.empty((9, self.ny, self.nx), dtype=t.float64, device=self.device)
        _check(load().lbm_populations(self._h, out.data_ptr(), self._s()), "lbm_populations")
        return out

    def history(self, max_rows: int = 4096) -> np.ndarray:
        buf = np.zeros((max_rows, 4))
        n = C.c_int(0)
        _check(load().lbm_history(self._h, buf.ctypes.data_as(C.POINTER(C.c_double)), max_rows, C.byref(n),
                                  self._s()), "lbm_history")
        return buf[: n.value]

    def state(self) -> tuple[int, int]:
        s, c = C.c_int64(0), C.c_int(0)
        _check(load().lbm_state(self._h, C.byref(s), C.byref(c)), "lbm_state")
        return s.value, c.value

    def current_buffer(self):
        return self.f[self.state()[1]]

    def save(self):
        t = self.torch
        out = t.empty(self.pop_bytes, dtype=t.uint8, device=self.device)
        _check(load().lbm_save(self._h, out.data_ptr(), self._s()), "lbm_save")
        return out, self.state()[0]

    def load_state(self, buf, step: int):
        _check(load().lbm_load(self._h, buf.data_ptr(), int(step), self._s()), "lbm_load")

    def enable_checkpointing(self, K: int, max_steps: int, overlap: bool = True):
        """Keep the state every K steps (up to max_steps) for lbm_adjoint; call before stepping.
        overlap: give lbm_adjoint a record buffer of two segments, so that it recomputes the next
        segment on a second stream while the transposed steps run over the current one."""
        t = self.torch
        slots = max(1, -(-int(max_steps) // int(K)))
        self._ckpt = t.empty(slots * self.pop_bytes, dtype=t.uint8, device=self.device)
        rec, adj = adjoint_layout(self.P, K)
        self._rec = t.empty(rec * (2 if overlap else 1), dtype=t.uint8, device=self.device)
        self._adj = t.empty(adj, dtype=t.uint8, device=self.device)
        _check(load().lbm_set_checkpointing(self._h, self._ckpt.data_ptr(), self._ckpt.numel(), int(K)),
               "lbm_set_checkpointing")

    def enable_recording(self, max_steps: int):
        """Keep every step's record (rho - rho_ref, j, psi) of the next max_steps steps in HBM so that
        lbm_adjoint runs no recomputation; call before stepping."""
        t = self.torch
        rec, adj = adjoint_layout(self.P, int(max_steps))
        self._recall = t.empty(rec, dtype=t.uint8, device=self.device)
        self._rec = None
        self._adj = t.empty(adj, dtype=t.uint8, device=self.device)
        _check(load().lbm_set_recording(self._h, self._recall.data_ptr(), self._recall.numel(), int(max_steps)),
               "lbm_set_recording")

    def adjoint(self, dL_drho, want_rho0: bool = False, dL_dux=None, dL_duy=None):
        """Gradient of a loss L(rho(T), u(T)) given dL/drho(T), dL/du_x(T), dL/du_y(T) [ny][nx] (None: zero):
        dict of GRAD_NAMES (+ 'rho0' field)."""
        t = self.torch
        shp = (self.ny, self.nx)
        g = self._dev(dL_drho, shp) if dL_drho is not None else None
        gx = self._dev(dL_dux, shp) if dL_dux is not None else None
        gy = self._dev(dL_duy, shp) if dL_duy is not None else None
        ptr = lambda a: a.data_ptr() if a is not None else None
        out = (C.c_double * 6)()
        r0 = t.empty(shp, dtype=t.float64, device=self.device) if want_rho0 else None
        rec = getattr(self, "_rec", None)
        _check(load().lbm_adjoint_fields(self._h, ptr(g), ptr(gx), ptr(gy), ptr(rec),
                                         rec.numel() if rec is not None else 0, self._adj.data_ptr(),
                                         self._adj.numel(), out, ptr(r0), self._s()),
               "lbm_adjoint_fields")
        res = dict(zip(GRAD_NAMES, list(out)))
        if r0 is not None:
            res["rho0"] = r0
        return res


# ---------------------------------------------------------------------------- batched lattices
class Batch:
    """B independent lattices advanced by one persistent launch (lbm_*_batched)."""

    def __init__(self, params, rho0s, device="cuda", stream=None):
        import torch

        self.torch = torch
        self.B = len(params)
        self.P = (LbmParams * self.B)(*params)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        pb, wb = C.c_size_t(0), C.c_size_t(0)
        offs = (C.c_int64 * (self.B + 1))()
        _check(load().lbm_batch_layout(self.B, self.P, C.byref(pb), C.byref(wb), offs), "lbm_batch_layout")
        self.offsets = [offs[i] for i in range(self.B + 1)]
        self.shapes = [(p.ny, p.nx) for p in params]
        self.f = [torch.empty(pb.value, dtype=torch.uint8, device=self.device) for _ in range(2)]
        self.ws = torch.zeros(wb.value, dtype=torch.uint8, device=self.device)
        packed = np.concatenate([np.ascontiguousarray(r, dtype=np.float64).reshape(-1) for r in rho0s])
        assert packed.size == self.offsets[-1]
        self._rho0 = torch.as_tensor(packed, device=self.device)
        h = C.c_void_p(0)
        _check(load().lbm_init_batched(C.byref(h), self.B, self.P, self.f[0].data_ptr(), self.f[1].data_ptr(),
                                       self.ws.data_ptr(), wb.value, self._rho0.data_ptr(), None, None,
                                       C.c_void_p(self.stream.cuda_stream)), "lbm_init_batched")
        self._h = h

    def step(self, n: int):
        _check(load().lbm_step_batched(self._h, int(n), C.c_void_p(self.stream.cuda_stream)), "lbm_step_batched")

    def set_mode(self, mode: int):
        """BATCH_AUTO, BATCH_PERSISTENT (one workgroup per lattice) or BATCH_GROUPED (a launch per step)."""
        _check(load().lbm_set_batch_mode(self._h, int(mode)), "lbm_set_batch_mode")

    def check(self):
        bad = C.c_int(-1)
        _check(load().lbm_status_batched(self._h, C.byref(bad), C.c_void_p(self.stream.cuda_stream)),
               "lbm_status_batched")

    def macros(self):
        t = self.torch
        n = self.offsets[-1]
        rho, ux, uy = (t.empty(n, dtype=t.float64, device=self.device) for _ in range(3))
        _check(load().lbm_macros_batched(self._h, rho.data_ptr(), ux.data_ptr(), uy.data_ptr(),
                                         C.c_void_p(self.stream.cuda_stream)), "lbm_macros_batched")
        out = []
        r, u, v = rho.cpu().numpy(), ux.cpu().numpy(), uy.cpu().numpy()
        for b, (ny, nx) in enumerate(self.shapes):
            sl = slice(self.offsets[b], self.offsets[b + 1])
            out.append({"rho": r[sl].reshape(ny, nx), "ux": u[sl].reshape(ny, nx), "uy": v[sl].reshape(ny, nx)})
        return out

    def close(self):
        if getattr(self, "_h", None):
            load().lbm_destroy_batched(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------- finite-difference reference solver
def make_fd_params(nx, ny, eos: LbmEos, h=1.0, dt=0.2, G=-1.0, eps=0.0, tau_e=1.0, tau_nu=1.0, var_tau=False,
                   tau_l=1.0, tau_v=1.0, rho_v_tau=None, rho_l_tau=None, walls=False) -> LbmFdParams:
    P = LbmFdParams()
    P.nx, P.ny, P.var_tau, P.walls = nx, ny, int(var_tau), int(walls)
    P.h, P.dt, P.G, P.eps, P.tau_e, P.tau_nu = h, dt, G, eps, tau_e, tau_nu
    P.tau_l, P.tau_v = tau_l, tau_v
    P.rho_v_tau = eos.rho_v if rho_v_tau is None else rho_v_tau
    P.rho_l_tau = eos.rho_l if rho_l_tau is None else rho_l_tau
    P.eos = eos
    return P


class FdSolver:
    """MacCormack finite-difference reference solver (lbm_fd_*) with state in one torch device buffer."""

    def __init__(self, P: LbmFdParams, rho0, u0=None, v0=None, device="cuda", stream=None):
        import torch

        self.torch = torch
        self.P = P
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nb = C.c_size_t(0)
        _check(load().lbm_fd_layout(C.byref(P), C.byref(nb)), "lbm_fd_layout")
        self.buf = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        shp = (P.ny, P.nx)
        f = [None if a is None else torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(shp),
                                                     device=self.device) for a in (rho0, u0, v0)]
        h = C.c_void_p(0)
        _check(load().lbm_fd_init(C.byref(h), C.byref(P), self.buf.data_ptr(), nb.value, f[0].data_ptr(),
                                  f[1].data_ptr() if f[1] is not None else None,
                                  f[2].data_ptr() if f[2] is not None else None, self._s()), "lbm_fd_init")
        self.torch.cuda.synchronize(self.device)
        self._h = h

    def _s(self):
        return C.c_void_p(self.stream.cuda_stream)

    def step(self, n: int):
        _check(load().lbm_fd_step(self._h, int(n), self._s()), "lbm_fd_step")

    def check(self):
        _check(load().lbm_fd_status(self._h, self._s()), "lbm_fd_status")

    def fields(self):
        t = self.torch
        shp = (self.P.ny, self.P.nx)
        out = [t.empty(shp, dtype=t.float64, device=self.device) for _ in range(3)]
        _check(load().lbm_fd_fields(self._h, *[o.data_ptr() for o in out], self._s()), "lbm_fd_fields")
        self.torch.cuda.synchronize(self.device)
        return out

    def close(self):
        if getattr(self, "_h", None):
            load().lbm_fd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
