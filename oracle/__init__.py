"""FP64 CPU oracle of the axisymmetric MRT lattice Boltzmann model (arXiv:1409.5929).

TEST INFRASTRUCTURE ONLY.  This package is the independent reference for the GPU
library: only the test suite, the package smoke check and the benchmark's
CPU-baseline leg may import it.  It shares no code with the GPU library, and
the GPU library never imports it.

The arithmetic lives in ``lbm_oracle.c`` (plain C, FP64, dense 9x9 moment
transforms); this module only marshals arguments through ctypes.  Each C
function cites the equations it follows.  ``build()`` compiles the C file with
gcc; ``Oracle`` wraps one lattice.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

SIDE = {"wall": 0, "axis": 1, "periodic": 2, "flow": 3}
THERM = {"fixed": 0, "adiabatic": 1, "flux": 2}


class _Params(ctypes.Structure):
    _fields_ = [
        ("nr", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("side_rmin", ctypes.c_int32), ("side_rmax", ctypes.c_int32), ("side_z", ctypes.c_int32),
        ("therm_rmin", ctypes.c_int32), ("therm_rmax", ctypes.c_int32), ("therm_z", ctypes.c_int32),
        ("r0", ctypes.c_double), ("L", ctypes.c_double), ("phi", ctypes.c_double),
        ("Da", ctypes.c_double), ("F_phi", ctypes.c_double), ("Ra", ctypes.c_double),
        ("Pr", ctypes.c_double), ("J", ctypes.c_double), ("lam", ctypes.c_double),
        ("Ma", ctypes.c_double), ("tau_nu", ctypes.c_double),
        ("accel_r", ctypes.c_double), ("accel_z", ctypes.c_double),
        ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double), ("s_q", ctypes.c_double),
        ("s_j", ctypes.c_double), ("s_nu", ctypes.c_double), ("src_printed", ctypes.c_int32),
        ("T_rmin", ctypes.c_double), ("T_rmax", ctypes.c_double),
        ("T_zmin", ctypes.c_double), ("T_zmax", ctypes.c_double),
        ("T_ref", ctypes.c_double), ("T_init", ctypes.c_double), ("delta_T", ctypes.c_double),
        ("flux_rmin", ctypes.c_double), ("flux_rmax", ctypes.c_double),
        ("flux_zlo", ctypes.c_double), ("flux_zhi", ctypes.c_double),
        ("u_in", ctypes.c_double),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle into ``liblbm_oracle.so`` next to its source."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.POINTER
    d = P(ctypes.c_double)
    lib.orc_create.restype = ctypes.c_void_p
    lib.orc_create.argtypes = [P(_Params), d, d]
    lib.orc_destroy.argtypes = [ctypes.c_void_p]
    lib.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.orc_time.restype = ctypes.c_long
    lib.orc_time.argtypes = [ctypes.c_void_p]
    lib.orc_macros.argtypes = [ctypes.c_void_p, d, d, d, d, d, P(ctypes.c_uint8)]
    lib.orc_snapshot.argtypes = [ctypes.c_void_p]
    lib.orc_snapshot.restype = None
    lib.orc_residual.restype = ctypes.c_int
    lib.orc_residual.argtypes = [ctypes.c_void_p, d]
    lib.orc_nusselt.argtypes = [ctypes.c_void_p, d, d]
    lib.orc_get_populations.argtypes = [ctypes.c_void_p, d, d]
    lib.orc_set_populations.argtypes = [ctypes.c_void_p, d, d]
    lib.orc_derived.argtypes = [ctypes.c_void_p, d]
    lib.orc_matrices.argtypes = [ctypes.c_void_p, d, d]
    lib.orc_node.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, d, d, d, d, d, d, d]
    lib.orc_pipe_nusselt.restype = ctypes.c_int
    lib.orc_pipe_nusselt.argtypes = [ctypes.c_void_p, ctypes.c_int, d, d]
    lib.orc_stream_function.restype = ctypes.c_double
    lib.orc_stream_function.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                        d, d]
    lib.orc_last_error.restype = ctypes.c_char_p
    lib.orc_threads.restype = ctypes.c_int
    _lib = lib
    return lib


DEFAULTS = dict(
    side_rmin="wall", side_rmax="wall", side_z="wall",
    therm_rmin="fixed", therm_rmax="fixed", therm_z="adiabatic",
    r0=1.0, L=1.0, phi=1.0, Da=1e8, F_phi=0.0, Ra=0.0, Pr=1.0, J=1.0, lam=1.0, Ma=0.1,
    tau_nu=0.0, accel_r=0.0, accel_z=0.0, s_e=1.1, s_eps=1.1, s_q=1.2, s_j=1.0, s_nu=0.0,
    src_printed=0,
    T_rmin=0.0, T_rmax=0.0, T_zmin=0.0, T_zmax=0.0, T_ref=0.0, T_init=0.0, delta_T=0.0,
    flux_rmin=0.0, flux_rmax=0.0, flux_zlo=-np.inf, flux_zhi=np.inf, u_in=0.0,
)


def _params(cfg: dict) -> _Params:
    c = dict(DEFAULTS)
    c.update({k: v for k, v in cfg.items() if k in DEFAULTS or k in ("nr", "nz")})
    p = _Params()
    for name, _ in _Params._fields_:
        v = c[name]
        if name.startswith("side_"):
            v = SIDE[v] if isinstance(v, str) else v
        elif name.startswith("therm_"):
            v = THERM[v] if isinstance(v, str) else v
        setattr(p, name, v)
    return p


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


class Oracle:
    """One lattice advanced by the FP64 oracle.

    ``cfg`` is a plain dict of the problem statement (grid, sides, porosity,
    Da, F_phi, Ra, Pr, J, lam, Ma, tau_nu, accelerations, rates, wall
    temperatures); ``phi_field`` is an optional [nz, nr] porosity array and
    ``init`` an optional [3, nz, nr] array of (u_z, u_r, T).
    """

    def __init__(self, cfg: dict, phi_field=None, init=None):
        lib = _load()
        self.cfg = dict(cfg)
        self.nr, self.nz = int(cfg["nr"]), int(cfg["nz"])
        self._p = _params(cfg)
        pf = None if phi_field is None else np.ascontiguousarray(phi_field, dtype=np.float64)
        ini = None if init is None else np.ascontiguousarray(init, dtype=np.float64)
        if pf is not None:
            assert pf.shape == (self.nz, self.nr)
        if ini is not None:
            assert ini.shape == (3, self.nz, self.nr)
        self._pf, self._ini = pf, ini
        h = lib.orc_create(ctypes.byref(self._p), _dptr(pf), _dptr(ini))
        if not h:
            raise ValueError("oracle: " + lib.orc_last_error().decode())
        self._h = ctypes.c_void_p(h)
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def t(self) -> int:
        return int(self._lib.orc_time(self._h))

    def step(self, n: int = 1):
        self._lib.orc_step(self._h, int(n))

    def macros(self) -> dict:
        shp = (self.nz, self.nr)
        out = {k: np.empty(shp) for k in ("uz", "ur", "p", "T", "rho")}
        mask = np.empty(shp, dtype=np.uint8)
        self._lib.orc_macros(self._h, _dptr(out["uz"]), _dptr(out["ur"]), _dptr(out["p"]),
                             _dptr(out["T"]), _dptr(out["rho"]),
                             mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        out["mask"] = mask
        return out

    def snapshot(self):
        """Keep the current u and T; residual() measures the change since."""
        self._lib.orc_snapshot(self._h)

    def residual(self):
        """Mean change per step since the snapshot (rms, scaled by Ma c_s and dT)."""
        out = np.empty(3)
        if self._lib.orc_residual(self._h, _dptr(out)) != 0:
            return None
        return dict(res_u=out[0], res_T=out[1], res=out[2])

    def nusselt(self):
        """(Nu_i, Nu_o): Eq. (42) on fixed-temperature walls, the heater mean of
        Eqs. (43)-(44) on flux walls."""
        a, b = ctypes.c_double(), ctypes.c_double()
        self._lib.orc_nusselt(self._h, ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value

    def pipe_nusselt(self, area: bool = False):
        """Local Nusselt number (Eq. 40) and bulk temperature at every column of
        a pipe (axis at r_min, wall at r_max): mixing-cup T_b, or with
        area=True the area mean as Eq. (41) is printed."""
        nu, tb = np.empty(self.nz), np.empty(self.nz)
        if self._lib.orc_pipe_nusselt(self._h, 1 if area else 0, _dptr(nu), _dptr(tb)) != 0:
            raise ValueError("pipe Nusselt numbers need an axis at r_min and a wall at r_max")
        return nu, tb

    def populations(self):
        f = np.empty((self.nz, self.nr, 9))
        g = np.empty((self.nz, self.nr, 5))
        self._lib.orc_get_populations(self._h, _dptr(f), _dptr(g))
        return f, g

    def set_populations(self, f, g):
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        assert f.shape == (self.nz, self.nr, 9) and g.shape == (self.nz, self.nr, 5)
        self._lib.orc_set_populations(self._h, _dptr(f), _dptr(g))

    def derived(self) -> dict:
        out = np.empty(6)
        self._lib.orc_derived(self._h, _dptr(out))
        return dict(zip(("tau_nu", "tau_T", "nu_e", "nu", "K_ref", "gbeta"), out.tolist()))

    def matrices(self):
        M = np.empty((9, 9))
        Mi = np.empty((9, 9))
        self._lib.orc_matrices(self._h, _dptr(M), _dptr(Mi))
        return M, Mi

    def node(self, r: float, phi: float, f, g):
        """One node in isolation: macro values, m^eq, S, post-collision f and g."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        macro, meq, S = np.empty(7), np.empty(9), np.empty(9)
        fo, go = np.empty(9), np.empty(5)
        self._lib.orc_node(self._h, float(r), float(phi), _dptr(f), _dptr(g), _dptr(macro),
                           _dptr(meq), _dptr(S), _dptr(fo), _dptr(go))
        return dict(rho=macro[0], ur=macro[1], uz=macro[2], T=macro[3], Ftr=macro[4],
                    Ftz=macro[5], a_r=macro[6], meq=meq, S=S, f_out=fo, g_out=go)


def stream_function(uz, r0: float, axis: bool = False):
    """Stokes stream function of a u_z field [nz, nr] with rows at r0 + j, zero
    on row 0 (an r_min wall) or, with axis=True, on the axis r = 0 (trapezoid
    rule); returns (psi, max |psi|)."""
    uz = np.ascontiguousarray(uz, dtype=np.float64)
    nz, nr = uz.shape
    psi = np.empty_like(uz)
    mx = _load().orc_stream_function(nr, nz, float(r0), 1 if axis else 0, _dptr(uz), _dptr(psi))
    return psi, float(mx)


def threads() -> int:
    return int(_load().orc_threads())
