"""TEST INFRASTRUCTURE ONLY -- ctypes binding and diagnostics of the FP64 CPU oracle.

The C side (``lbm_oracle.c``) holds the method; this module marshals arguments and
adds the paper's post-processing: the vapor-density error (Eq. DensityError), the
interface width (Sec. III.A, 0.01 < (rho-rho_v)/(rho_l-rho_v) < 0.99), the surface
tension (Eq. SurfaceTension, fourth-order central difference + Simpson) and the
convergence criterion of Sec. III.A.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_SRC_FD = os.path.join(_HERE, "fd_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")
# the same source with its node loops split over rows by OpenMP (-DOR_OMP): same bits, more cores
_LIB_OMP = os.path.join(_HERE, "liblbm_oracle_omp.so")
_lock = threading.Lock()
_lib = None
_lib_omp = None

OR_OK, OR_EINVAL, OR_EUNSTABLE, OR_ENOROOT = 0, -1, -2, -5
BASE_CS, BASE_PR = 0, 1
SHAPE_NONE, SHAPE_SMOOTH, SHAPE_MODSMOOTH, SHAPE_PENG = 0, 1, 2, 3
FORCING_GUO, FORCING_LI = 0, 1

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


class OrEos(C.Structure):
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


class OrParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("walls", C.c_int), ("forcing", C.c_int),
        ("var_tau", C.c_int), ("pad_", C.c_int),
        ("rho_wall_lo", C.c_double), ("rho_wall_hi", C.c_double),
        ("G", C.c_double), ("sigma", C.c_double),
        ("tau", C.c_double * 9),
        ("tau_l", C.c_double), ("tau_v", C.c_double),
        ("rho_v_tau", C.c_double), ("rho_l_tau", C.c_double),
        ("eos", OrEos),
    ]


class OrFdParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("var_tau", C.c_int), ("walls", C.c_int),
        ("h", C.c_double), ("dt", C.c_double), ("G", C.c_double), ("eps", C.c_double),
        ("tau_e", C.c_double), ("tau_nu", C.c_double),
        ("tau_l", C.c_double), ("tau_v", C.c_double), ("rho_v_tau", C.c_double), ("rho_l_tau", C.c_double),
        ("psi_wall", C.c_double),
        ("eos", OrEos),
    ]


def _stale(path: str) -> bool:
    return not os.path.exists(path) or os.path.getmtime(path) < max(
        os.path.getmtime(_SRC), os.path.getmtime(_SRC_FD), os.path.getmtime(os.path.join(_HERE, "lbm_oracle.h")))


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no vector intrinsics), single-threaded and with
    OpenMP over the rows of each node loop."""
    with _lock:
        for out, extra in ((_LIB, []), (_LIB_OMP, ["-DOR_OMP", "-fopenmp"])):
            if force or _stale(out):
                tmp = out + ".tmp%d" % os.getpid()
                subprocess.check_call(
                    ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", *extra, "-o", tmp, _SRC, _SRC_FD, "-lm"]
                )
                os.replace(tmp, out)
    return _LIB


def lib(omp: bool = False):
    """The single-threaded oracle library, or (omp=True) its OpenMP build."""
    global _lib, _lib_omp
    if (_lib_omp if omp else _lib) is None:
        build()
        L = C.CDLL(_LIB_OMP if omp else _LIB)
        d, i, p = C.c_double, C.c_int, C.c_void_p
        dp = C.POINTER(C.c_double)
        L.or_eos_build.argtypes = [C.POINTER(OrEos), d, dp]
        L.or_eos_build.restype = i
        L.or_eos_set_knots.argtypes = [C.POINTER(OrEos), d, d, d, d]
        L.or_eos_set_knots.restype = i
        for name in ("or_base_p", "or_base_dp", "or_eos_p", "or_eos_dp"):
            getattr(L, name).argtypes = [C.POINTER(OrEos), d]
            getattr(L, name).restype = d
        L.or_cs_critical_eta.restype = d
        L.or_maxwell_residual.argtypes = [C.POINTER(OrEos), d, d, d, i]
        L.or_maxwell_residual.restype = d
        L.or_mech_residual.argtypes = [C.POINTER(OrEos), d, d]
        L.or_mech_residual.restype = d
        L.or_fd_new.argtypes = [C.POINTER(OrFdParams)]
        L.or_fd_new.restype = p
        L.or_fd_free.argtypes = [p]
        L.or_fd_set.argtypes = [p, dp, dp, dp]
        L.or_fd_get.argtypes = [p, dp, dp, dp]
        L.or_fd_run.argtypes = [p, C.c_longlong]
        L.or_fd_run.restype = i
        L.or_lattice_new.argtypes = [C.POINTER(OrParams)]
        L.or_lattice_new.restype = p
        L.or_lattice_free.argtypes = [p]
        L.or_init_eq.argtypes = [p, dp, dp, dp]
        L.or_set_f.argtypes = [p, dp]
        L.or_get_f.argtypes = [p, dp]
        L.or_run.argtypes = [p, C.c_longlong]
        L.or_run.restype = i
        L.or_run_window.argtypes = [p, C.c_longlong]
        L.or_run_window.restype = i
        L.or_fail_step.argtypes = [p]
        L.or_fail_step.restype = C.c_longlong
        L.or_macros.argtypes = [p, dp, dp, dp, dp, dp, dp, dp]
        L.or_macros.restype = i
        L.or_collide_node.argtypes = [C.POINTER(OrParams), dp, d, d, d, d, d, dp]
        L.or_feq.argtypes = [d, d, d, dp]
        L.or_force_tilde_field.argtypes = [i, i, dp, i, d, d, d, dp, dp]
        L.or_matrix.argtypes = [dp, dp]
        L.or_threads.restype = i
        if omp:
            _lib_omp = L
        else:
            _lib = L
    return _lib_omp if omp else _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleError(RuntimeError):
    pass


# ---------------------------------------------------------------------------
# thermodynamics
# ---------------------------------------------------------------------------
def make_eos(base=BASE_CS, shape=SHAPE_NONE, a=0.5, b=4.0, R=1.0, omega=0.344, Tr=0.7,
             scale=1.0, alpha=1.0, k_vap=1.0, r_theta=0.0) -> OrEos:
    e = OrEos()
    e.base, e.shape = base, shape
    e.a, e.b, e.R, e.omega, e.Tr = a, b, R, omega, Tr
    e.scale, e.alpha, e.k_vap, e.r_theta = scale, alpha, k_vap, r_theta
    return e


def eos_build(e: OrEos, G: float = -1.0) -> tuple[OrEos, float]:
    """Host precompute: Tc, Maxwell coexistence, shaped loop, eps and sigma = -eps/(16G)."""
    s = C.c_double(0.0)
    st = lib().or_eos_build(C.byref(e), G, C.byref(s))
    if st != OR_OK:
        raise OracleError("or_eos_build failed with status %d" % st)
    return e, s.value


def eos_set_knots(e: OrEos, rho_max: float, p_max: float, rho_min: float, p_min: float) -> OrEos:
    """Copy of a built Smooth loop with its four knots replaced and both ellipses refitted."""
    out = OrEos()
    C.memmove(C.byref(out), C.byref(e), C.sizeof(OrEos))
    st = lib().or_eos_set_knots(C.byref(out), rho_max, p_max, rho_min, p_min)
    if st != OR_OK:
        raise OracleError("or_eos_set_knots failed with status %d" % st)
    return out


def eos_p(e: OrEos, rho) -> np.ndarray:
    L = lib()
    r = np.atleast_1d(np.asarray(rho, dtype=np.float64))
    return np.array([L.or_eos_p(C.byref(e), float(x)) for x in r])


def eos_dp(e: OrEos, rho) -> np.ndarray:
    L = lib()
    r = np.atleast_1d(np.asarray(rho, dtype=np.float64))
    return np.array([L.or_eos_dp(C.byref(e), float(x)) for x in r])


def base_p(e: OrEos, rho) -> np.ndarray:
    L = lib()
    r = np.atleast_1d(np.asarray(rho, dtype=np.float64))
    return np.array([L.or_base_p(C.byref(e), float(x)) for x in r])


def base_dp(e: OrEos, rho) -> np.ndarray:
    L = lib()
    r = np.atleast_1d(np.asarray(rho, dtype=np.float64))
    return np.array([L.or_base_dp(C.byref(e), float(x)) for x in r])


def maxwell_residual(e: OrEos, p0: float, lo: float, hi: float, shaped: bool) -> float:
    return lib().or_maxwell_residual(C.byref(e), p0, lo, hi, int(shaped))


def mech_residual(e: OrEos, eps: float, G: float = -1.0) -> float:
    return lib().or_mech_residual(C.byref(e), eps, G)


def cs_critical_eta() -> float:
    return lib().or_cs_critical_eta()


# ---------------------------------------------------------------------------
# lattice
# ---------------------------------------------------------------------------
def make_params(nx, ny, eos: OrEos, G=-1.0, sigma=0.0, forcing=FORCING_LI, tau=None,
                walls=False, rho_wall_lo=0.0, rho_wall_hi=0.0, var_tau=False, tau_l=1.0,
                tau_v=1.0, rho_v_tau=None, rho_l_tau=None) -> OrParams:
    P = OrParams()
    P.nx, P.ny, P.walls, P.forcing, P.var_tau = nx, ny, int(walls), forcing, int(var_tau)
    P.rho_wall_lo, P.rho_wall_hi = rho_wall_lo, rho_wall_hi
    P.G, P.sigma = G, sigma
    t = [1.0] * 9 if tau is None else list(tau)
    for k in range(9):
        P.tau[k] = t[k]
    P.tau_l, P.tau_v = tau_l, tau_v
    P.rho_v_tau = eos.rho_v if rho_v_tau is None else rho_v_tau
    P.rho_l_tau = eos.rho_l if rho_l_tau is None else rho_l_tau
    P.eos = eos
    return P


def make_fd_params(nx, ny, eos: OrEos, h=1.0, dt=0.2, G=-1.0, eps=0.0, tau_e=1.0, tau_nu=1.0, var_tau=False,
                   tau_l=1.0, tau_v=1.0, rho_v_tau=None, rho_l_tau=None, walls=False) -> OrFdParams:
    """walls: the appendix's wall layers in y, with psi_l = psi(rho_l) of the EOS in Eq. B2."""
    P = OrFdParams()
    P.nx, P.ny, P.var_tau, P.walls = nx, ny, int(var_tau), int(walls)
    if walls:
        q = 2.0 * (eos_p(eos, eos.rho_l)[0] - eos.rho_l / 3.0) / G
        P.psi_wall = float(np.sqrt(q)) if q > 0 else 0.0
    P.h, P.dt, P.G, P.eps, P.tau_e, P.tau_nu = h, dt, G, eps, tau_e, tau_nu
    P.tau_l, P.tau_v = tau_l, tau_v
    P.rho_v_tau = eos.rho_v if rho_v_tau is None else rho_v_tau
    P.rho_l_tau = eos.rho_l if rho_l_tau is None else rho_l_tau
    P.eos = eos
    return P


class FdSolver:
    """Finite-difference reference solver (MacCormack): periodic in x; in y periodic or the appendix wall layers."""

    def __init__(self, P: OrFdParams):
        self.P = P
        self._h = lib().or_fd_new(C.byref(P))
        if not self._h:
            raise OracleError("or_fd_new rejected the parameters")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_fd_free(self._h)
            self._h = None

    def set(self, rho, u=None, v=None):
        shp = (self.P.ny, self.P.nx)
        r = np.ascontiguousarray(rho, dtype=np.float64).reshape(shp)
        uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(shp)
        vv = None if v is None else np.ascontiguousarray(v, dtype=np.float64).reshape(shp)
        lib().or_fd_set(self._h, _ptr(r), _ptr(uu), _ptr(vv))

    def get(self):
        shp = (self.P.ny, self.P.nx)
        r, u, v = np.empty(shp), np.empty(shp), np.empty(shp)
        lib().or_fd_get(self._h, _ptr(r), _ptr(u), _ptr(v))
        return r, u, v

    def run(self, n: int):
        st = lib().or_fd_run(self._h, int(n))
        if st != OR_OK:
            raise OracleError("FD solver unstable (psi^2 < 0 or non-positive density)")


class Lattice:
    """FP64 oracle lattice; populations f_i(t, x) stored [9][ny][nx].

    omp=True runs the OpenMP build (rows of each node loop split over threads; the same
    bits as the single-threaded build)."""

    def __init__(self, P: OrParams, omp: bool = False):
        self.P = P
        self.nx, self.ny = P.nx, P.ny
        self._L = lib(omp)
        self._h = self._L.or_lattice_new(C.byref(P))
        if not self._h:
            raise OracleError("invalid lattice size")
        self.step = 0

    @property
    def threads(self) -> int:
        """Threads a time step of this lattice uses (1 for the single-threaded build)."""
        return int(self._L.or_threads())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.or_lattice_free(h)
            self._h = None

    def init_eq(self, rho, ux=None, uy=None):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.ny, self.nx)
        ux = None if ux is None else np.ascontiguousarray(ux, dtype=np.float64).reshape(self.ny, self.nx)
        uy = None if uy is None else np.ascontiguousarray(uy, dtype=np.float64).reshape(self.ny, self.nx)
        self._L.or_init_eq(self._h, _ptr(rho), _ptr(ux), _ptr(uy))
        self.step = 0

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(9, self.ny, self.nx)
        self._L.or_set_f(self._h, _ptr(f))

    def get_f(self) -> np.ndarray:
        f = np.empty((9, self.ny, self.nx))
        self._L.or_get_f(self._h, _ptr(f))
        return f

    def run(self, nsteps: int) -> None:
        st = self._L.or_run(self._h, int(nsteps))
        if st != OR_OK:
            raise OracleError("oracle run unstable at step %d" % self._L.or_fail_step(self._h))
        self.step += int(nsteps)

    def run_window(self, nsteps: int) -> None:
        """Steps of a periodic window cut from a larger lattice: nodes the cut makes unphysical
        get NaN psi instead of stopping the run; NaN then spreads two nodes per step at most."""
        self._L.or_run_window(self._h, int(nsteps))
        self.step += int(nsteps)

    def macros(self) -> dict:
        shp = (self.ny, self.nx)
        out = {k: np.empty(shp) for k in ("rho", "ux", "uy", "psi", "p", "Fx", "Fy")}
        st = self._L.or_macros(self._h, *[_ptr(out[k]) for k in ("rho", "ux", "uy", "psi", "p", "Fx", "Fy")])
        if st != OR_OK:
            raise OracleError("psi not real")
        return out


def collide_node(P: OrParams, f, Fx, Fy, psi, Ftx, Fty) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty(9)
    lib().or_collide_node(C.byref(P), _ptr(f), Fx, Fy, psi, Ftx, Fty, _ptr(out))
    return out


def feq(rho, ux, uy) -> np.ndarray:
    out = np.empty(9)
    lib().or_feq(rho, ux, uy, _ptr(out))
    return out


def force_tilde_field(psi, G=-1.0, walls=False, psi_lo=0.0, psi_hi=0.0):
    """F~ = F/psi(x) of Eq. ShanChenForce on a given psi[ny][nx] field."""
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    ny, nx = psi.shape
    fx, fy = np.empty_like(psi), np.empty_like(psi)
    lib().or_force_tilde_field(nx, ny, _ptr(psi), int(walls), psi_lo, psi_hi, G, _ptr(fx), _ptr(fy))
    return fx, fy


def matrices() -> tuple[np.ndarray, np.ndarray]:
    M = np.empty(81)
    Mi = np.empty(81)
    lib().or_matrix(_ptr(M), _ptr(Mi))
    return M.reshape(9, 9), Mi.reshape(9, 9)


# ---------------------------------------------------------------------------
# diagnostics (Sec. III.A, Sec. IV)
# ---------------------------------------------------------------------------
def density_error(rho_v_sim: float, rho_v_maxwell: float) -> float:
    """Eq. DensityError, in percent."""
    return 100.0 * (rho_v_sim - rho_v_maxwell) / rho_v_maxwell


def convergence_residual(rho_now: np.ndarray, rho_prev: np.ndarray) -> float:
    """Sec. III.A: sum |rho(t) - rho(t-100)| / sum |rho(t)|."""
    return float(np.abs(rho_now - rho_prev).sum() / np.abs(rho_now).sum())


def interface_cells(profile: np.ndarray, rho_v: float, rho_l: float) -> int:
    """Number of nodes of a 1-D profile inside 0.01 < (rho-rho_v)/(rho_l-rho_v) < 0.99."""
    phi = (profile - rho_v) / (rho_l - rho_v)
    return int(np.count_nonzero((phi > 0.01) & (phi < 0.99)))


def surface_tension_planar(psi_y: np.ndarray, G: float = -1.0) -> float:
    """gamma = -(G c^4/6) int (dpsi/dy)^2 dy across one interface of the 2-interface planar profile."""
    psi = np.asarray(psi_y, dtype=np.float64)
    n = psi.size
    d = (-np.roll(psi, -2) + 8 * np.roll(psi, -1) - 8 * np.roll(psi, 1) + np.roll(psi, 2)) / 12.0
    g = d * d
    # half period: from the vapor centre (y = 0) to the liquid centre (y = n/2)
    half = n // 2
    seg = g[: half + 1]
    m = seg.size - 1
    if m % 2:
        raise ValueError("need an even number of intervals")
    w = np.ones(m + 1)
    w[1:-1:2] = 4
    w[2:-1:2] = 2
    integral = (w * seg).sum() / 3.0
    return -G / 6.0 * integral


def run_planar(eos: OrEos, G=-1.0, sigma=None, forcing=FORCING_LI, ny=200, nx=2, W=10.0,
               check_every=100, tol=1e-6, max_steps=400000, tau=None):
    """Planar liquid-vapor interface of Sec. III.A run to the convergence criterion.

    Returns a dict with the measured rho_v (vapor-band centre), rho_l (liquid-band centre),
    the vapor error E (Eq. DensityError), the interface cell count, gamma and the step count.
    """
    from lbm_inputs import planar_density

    if sigma is None:
        sigma = -eos.eps / (16.0 * G)
    P = make_params(nx, ny, eos, G=G, sigma=sigma, forcing=forcing, tau=tau)
    L = Lattice(P)
    rho0 = planar_density(nx, ny, eos.rho_v, eos.rho_l, W=W, axis=1)
    L.init_eq(rho0)
    prev = L.macros()["rho"]
    steps = 0
    res = 1.0
    while steps < max_steps:
        L.run(check_every)
        steps += check_every
        cur = L.macros()["rho"]
        res = convergence_residual(cur, prev)
        prev = cur
        if res < tol:
            break
    m = L.macros()
    prof = m["rho"][:, 0]
    rv = float(prof[0])
    rl = float(prof[ny // 2])
    half = prof[: ny // 2 + 1]
    return {
        "rho_v": rv,
        "rho_l": rl,
        "E": density_error(rv, eos.rho_v),
        "width": interface_cells(half, rv, rl),
        "gamma": surface_tension_planar(m["psi"][:, 0], G),
        "steps": steps,
        "residual": res,
        "fields": m,
    }
