"""Python binding of the lbm_axi C-ABI (argument marshalling only).

Every step of the method runs in the HIP kernels of ``liblbm_axi.so``; this
module packs problem dictionaries into ``lbm_axi_params``, hands host arrays
and a HIP stream to the library and unpacks what it returns.  PyTorch, when
present, only supplies the stream and device buffers; it is imported before
the library is loaded so that both share one HIP runtime.

The entry points mirror ``include/lbm_axi.h``: lbm_axi_create is
Lattice(...), lbm_axi_default_params fills every parameter a problem
dictionary leaves out, and every other lbm_axi_<name> is Lattice.<name>
(macros is also available as fields, destroy as close; macros with device
outputs is fields_device).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm_axi.so")

SIDE = {"wall": 0, "axis": 1, "periodic": 2, "flow": 3}
THERM = {"fixed": 0, "adiabatic": 1, "flux": 2}
STORAGE = {"fp32": 0, "fp16": 1, "bf16": 2}
RUN_STATE = {0: "running", 1: "converged", 2: "diverged", 3: "stalled"}


class Params(ctypes.Structure):
    """ctypes image of ``lbm_axi_params`` (field order and types as in the header)."""

    _fields_ = [
        ("nr", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("side_rmin", ctypes.c_int32), ("side_rmax", ctypes.c_int32), ("side_z", ctypes.c_int32),
        ("therm_rmin", ctypes.c_int32), ("therm_rmax", ctypes.c_int32), ("therm_z", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("storage_shift", ctypes.c_int32),
        ("check_interval", ctypes.c_int32), ("src_printed", ctypes.c_int32),
        ("r0", ctypes.c_double), ("L", ctypes.c_double), ("phi", ctypes.c_double),
        ("Da", ctypes.c_double), ("F_phi", ctypes.c_double), ("Ra", ctypes.c_double),
        ("Pr", ctypes.c_double), ("J", ctypes.c_double), ("lambda_", ctypes.c_double),
        ("sigma", ctypes.c_double), ("Ma", ctypes.c_double), ("tau_nu", ctypes.c_double),
        ("accel_r", ctypes.c_double), ("accel_z", ctypes.c_double),
        ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double), ("s_q", ctypes.c_double),
        ("s_j", ctypes.c_double),
        ("T_rmin", ctypes.c_double), ("T_rmax", ctypes.c_double), ("T_zmin", ctypes.c_double),
        ("T_zmax", ctypes.c_double), ("T_ref", ctypes.c_double), ("T_init", ctypes.c_double),
        ("delta_T", ctypes.c_double), ("tol", ctypes.c_double), ("max_steps", ctypes.c_int64),
        ("flux_rmin", ctypes.c_double), ("flux_rmax", ctypes.c_double),
        ("flux_zlo", ctypes.c_double), ("flux_zhi", ctypes.c_double),
        ("u_in", ctypes.c_double), ("tail_tol", ctypes.c_double),
    ]


_ALIASES = {"lam": "lambda_", "lambda": "lambda_"}


def make_params(cfg: dict, storage: str = "fp32", check_interval: int = 100, tol: float = 0.0,
                max_steps: int = 0, storage_shift: int = 0, tail_tol: float = 0.0) -> Params:
    """Pack a problem dictionary (see ``lbm_inputs``) into ``lbm_axi_params``."""
    p = Params()
    lib = _load()
    lib.lbm_axi_default_params(ctypes.byref(p))
    for key, val in cfg.items():
        name = _ALIASES.get(key, key)
        if name.startswith("side_"):
            val = SIDE[val] if isinstance(val, str) else int(val)
        elif name.startswith("therm_"):
            val = THERM[val] if isinstance(val, str) else int(val)
        if not hasattr(p, name):
            continue
        setattr(p, name, val)
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.storage_shift = int(storage_shift)
    p.check_interval = int(check_interval)
    p.tol = float(cfg.get("tol", tol))  # a problem may carry its own stopping rule
    p.max_steps = int(cfg.get("max_steps", max_steps))
    p.tail_tol = float(cfg.get("tail_tol", tail_tol))
    return p


def derived(cfg: dict) -> dict:
    """tau_nu, tau_T (Eq. 39), nu_e (Eq. 31), nu, K (Eq. 9), g beta and
    alpha_e = c_sT^2 tau_T of a problem, as the library derives them (no device
    needed)."""
    p = make_params(cfg)
    out = (ctypes.c_double * 7)()
    _check(_load().lbm_axi_derived(ctypes.byref(p), out))
    return dict(zip(("tau_nu", "tau_T", "nu_e", "nu", "K_ref", "gbeta", "alpha_e"), list(out)))


_lib = None


def _load():
    """Load the HIP library; raise if it has not been built (no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    try:  # share torch's HIP runtime when torch is present
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() (or "
                           "python -m paper_1409_5929_amd.build) first")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    fp = P(ctypes.c_float)
    lib.lbm_axi_default_params.argtypes = [P(Params)]
    lib.lbm_axi_default_params.restype = None
    lib.lbm_axi_create.argtypes = [P(Params), ctypes.c_int32, P(fp), P(fp), ctypes.c_void_p,
                                   P(ctypes.c_void_p)]
    lib.lbm_axi_create.restype = ctypes.c_int
    lib.lbm_axi_step.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.lbm_axi_step.restype = ctypes.c_int
    lib.lbm_axi_macros.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_int32]
    lib.lbm_axi_macros.restype = ctypes.c_int
    lib.lbm_axi_stream_function_static.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                                   ctypes.c_void_p]
    lib.lbm_axi_stream_function_static.restype = ctypes.c_int
    lib.lbm_axi_pattern_bandwidth.argtypes = [ctypes.c_void_p, ctypes.c_int32, P(ctypes.c_double)]
    lib.lbm_axi_pattern_bandwidth.restype = ctypes.c_int
    lib.lbm_axi_derived.argtypes = [P(Params), P(ctypes.c_double)]
    lib.lbm_axi_derived.restype = ctypes.c_int
    lib.lbm_axi_density_deviation.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                              ctypes.c_int32]
    lib.lbm_axi_density_deviation.restype = ctypes.c_int
    lib.lbm_axi_residual.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]
    lib.lbm_axi_residual.restype = ctypes.c_int
    lib.lbm_axi_info.argtypes = [ctypes.c_void_p, ctypes.c_int32, P(ctypes.c_int64)]
    lib.lbm_axi_info.restype = ctypes.c_int
    lib.lbm_axi_stream_function.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            P(ctypes.c_double), ctypes.c_int32]
    lib.lbm_axi_stream_function.restype = ctypes.c_int
    lib.lbm_axi_pipe_nusselt.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_void_p]
    lib.lbm_axi_pipe_nusselt.restype = ctypes.c_int
    lib.lbm_axi_set_timing.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.lbm_axi_set_timing.restype = ctypes.c_int
    lib.lbm_axi_kernel_time.argtypes = [ctypes.c_void_p, P(ctypes.c_double), P(ctypes.c_int64)]
    lib.lbm_axi_kernel_time.restype = ctypes.c_int
    lib.lbm_axi_set_tiles.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]
    lib.lbm_axi_set_tiles.restype = ctypes.c_int
    lib.lbm_axi_lane_bandwidth.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
    lib.lbm_axi_lane_bandwidth.restype = ctypes.c_int
    lib.lbm_axi_set_wall_lanes.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.lbm_axi_set_wall_lanes.restype = ctypes.c_int
    lib.lbm_axi_set_storage.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]
    lib.lbm_axi_set_storage.restype = ctypes.c_int
    lib.lbm_axi_set_graph.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.lbm_axi_set_graph.restype = ctypes.c_int
    lib.lbm_axi_compact.argtypes = [ctypes.c_void_p, P(ctypes.c_int32)]
    lib.lbm_axi_compact.restype = ctypes.c_int
    lib.lbm_axi_autotune.argtypes = [ctypes.c_void_p, ctypes.c_int32, P(ctypes.c_int32),
                                     P(ctypes.c_int32), P(ctypes.c_double)]
    lib.lbm_axi_autotune.restype = ctypes.c_int
    lib.lbm_axi_sync.argtypes = [ctypes.c_void_p]
    lib.lbm_axi_sync.restype = ctypes.c_int
    lib.lbm_axi_destroy.argtypes = [ctypes.c_void_p]
    lib.lbm_axi_destroy.restype = None
    lib.lbm_axi_last_error.argtypes = []
    lib.lbm_axi_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


class LbmError(RuntimeError):
    pass


def _check(rc: int):
    if rc != 0:
        raise LbmError(f"lbm_axi error {rc}: {_load().lbm_axi_last_error().decode()}")


def _current_stream():
    try:
        import torch

        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return ctypes.c_void_p(None)


class Lattice:
    """One handle holding one or several instances.

    ``cfg`` is a problem dict or a list of them; ``phi`` an optional [nz, nr]
    porosity array (or a list, entries may be None); ``init`` an optional
    [3, nz, nr] array of (u_z, u_r, T) (or a list).  ``stream`` is a raw
    hipStream_t value; by default torch's current stream.
    """

    def __init__(self, cfg, phi=None, init=None, storage="fp32", check_interval=100,
                 tol=0.0, max_steps=0, storage_shift=0, stream=None, tail_tol=0.0):
        lib = _load()
        cfgs = list(cfg) if isinstance(cfg, (list, tuple)) else [cfg]
        n = len(cfgs)
        phis = list(phi) if isinstance(phi, (list, tuple)) else [phi] * (1 if n == 1 else 0)
        inits = list(init) if isinstance(init, (list, tuple)) else [init] * (1 if n == 1 else 0)
        if not phis:
            phis = [None] * n
        if not inits:
            inits = [None] * n
        if len(phis) != n or len(inits) != n:
            raise ValueError("phi and init must be given per instance (or once for a single instance)")
        self.shapes = [(int(c["nz"]), int(c["nr"])) for c in cfgs]
        self.cfgs = cfgs
        arr = (Params * n)()
        for i, c in enumerate(cfgs):
            arr[i] = make_params(c, storage, check_interval, tol, max_steps, storage_shift, tail_tol)
        keep = []
        fp = ctypes.POINTER(ctypes.c_float)
        phi_ptrs = (fp * n)()
        init_ptrs = (fp * n)()
        for i in range(n):
            nz, nr = self.shapes[i]
            if phis[i] is not None:
                a = np.ascontiguousarray(phis[i], dtype=np.float32)
                if a.shape != (nz, nr):
                    raise ValueError(f"porosity field {i} has shape {a.shape}, expected {(nz, nr)}")
                keep.append(a)
                phi_ptrs[i] = a.ctypes.data_as(fp)
            if inits[i] is not None:
                a = np.ascontiguousarray(inits[i], dtype=np.float32)
                if a.shape != (3, nz, nr):
                    raise ValueError(f"start fields {i} have shape {a.shape}, expected {(3, nz, nr)}")
                keep.append(a)
                init_ptrs[i] = a.ctypes.data_as(fp)
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(stream) if stream is not None else _current_stream()
        _check(lib.lbm_axi_create(arr, n, phi_ptrs, init_ptrs, st, ctypes.byref(h)))
        self._stream = st.value or 0
        self._h = h
        self._lib = lib
        self.n_inst = n

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.lbm_axi_destroy(self._h)
            self._h = ctypes.c_void_p()

    destroy = close

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def step(self, n: int = 1):
        _check(self._lib.lbm_axi_step(self._h, int(n)))

    def sync(self):
        _check(self._lib.lbm_axi_sync(self._h))

    def fields(self, inst: int = 0, drho: bool = True) -> dict:
        """Host copies of u_z, u_r, p, T (float32), the node classes (uint8) and,
        with drho=True, the density deviation rho - 1 (float32, "drho")."""
        nz, nr = self.shapes[inst]
        out = {k: np.empty((nz, nr), dtype=np.float32) for k in ("uz", "ur", "p", "T")}
        mask = np.empty((nz, nr), dtype=np.uint8)
        _check(self._lib.lbm_axi_macros(self._h, int(inst), out["uz"].ctypes.data,
                                        out["ur"].ctypes.data, out["p"].ctypes.data,
                                        out["T"].ctypes.data, mask.ctypes.data, 0))
        out["mask"] = mask
        if drho:
            out["drho"] = self.density_deviation(inst)
        return out

    def density_deviation(self, inst: int = 0) -> np.ndarray:
        """rho - 1 at every node as a host [nz, nr] float32 array."""
        nz, nr = self.shapes[inst]
        out = np.empty((nz, nr), dtype=np.float32)
        _check(self._lib.lbm_axi_density_deviation(self._h, int(inst), out.ctypes.data, 0))
        return out

    macros = fields

    def fields_device(self, inst: int = 0) -> dict:
        """u_z, u_r, p, T as torch device tensors, written on the handle's
        stream.  The tensors belong to torch's current stream: unless the
        handle runs on that very stream, this waits for the handle's stream
        before returning, so that neither a reader nor torch's allocator sees
        them before they are written."""
        import torch

        nz, nr = self.shapes[inst]
        out = {k: torch.empty((nz, nr), dtype=torch.float32, device="cuda")
               for k in ("uz", "ur", "p", "T")}
        _check(self._lib.lbm_axi_macros(self._h, int(inst), out["uz"].data_ptr(),
                                        out["ur"].data_ptr(), out["p"].data_ptr(),
                                        out["T"].data_ptr(), None, 1))
        # A zero stream value means the library created its own stream.
        if self._stream == 0 or self._stream != (torch.cuda.current_stream().cuda_stream or 0):
            self.sync()
        return out

    def stream_function(self, inst: int = 0, field: bool = True):
        """Stokes stream function of one instance (lattice units, zero on the r_min
        wall or on the axis) as a host [nz, nr] float32 array (None with
        field=False) and max |psi|."""
        nz, nr = self.shapes[inst]
        psi = np.empty((nz, nr), dtype=np.float32) if field else None
        mx = ctypes.c_double()
        _check(self._lib.lbm_axi_stream_function(self._h, int(inst),
                                                 psi.ctypes.data if field else None,
                                                 ctypes.byref(mx), 0))
        return psi, mx.value

    def stream_function_static(self, inst: int = 0, psi=None, psi_absmax=None):
        """The stream function written into caller device memory without any
        allocation: psi a float32 [nz, nr] device tensor (or None), psi_absmax a
        float64 device tensor of one element (or None); written on the
        handle's stream."""
        import torch

        nz, nr = self.shapes[int(inst)]
        # the library writes nz nr floats and one double through these pointers
        for t, dtype, n, what in ((psi, torch.float32, nz * nr, "psi"), (psi_absmax, torch.float64, 1, "psi_absmax")):
            if t is None:
                continue
            if t.dtype != dtype or t.numel() != n or not t.is_contiguous():
                raise ValueError(f"{what}: expected a contiguous {dtype} tensor of {n} elements")
            if not t.is_cuda:
                raise ValueError(f"{what}: expected device memory")
        _check(self._lib.lbm_axi_stream_function_static(
            self._h, int(inst), None if psi is None else psi.data_ptr(),
            None if psi_absmax is None else psi_absmax.data_ptr()))

    def pipe_nusselt(self, inst: int = 0, area: bool = False):
        """Local Nusselt number (Eq. 40) and bulk temperature at every column of
        a pipe instance, as two float64 arrays of length nz: mixing-cup T_b, or
        with area=True the area mean as Eq. (41) is printed."""
        nz, _ = self.shapes[inst]
        nu, tb = np.empty(nz), np.empty(nz)
        _check(self._lib.lbm_axi_pipe_nusselt(self._h, int(inst), 1 if area else 0,
                                              nu.ctypes.data, tb.ctypes.data))
        return nu, tb

    def residual(self) -> dict:
        n = self.n_inst
        res, nui, nuo = np.empty(n), np.empty(n), np.empty(n)
        st = np.empty(n, dtype=np.int32)
        _check(self._lib.lbm_axi_residual(self._h, res.ctypes.data, nui.ctypes.data,
                                          nuo.ctypes.data, st.ctypes.data))
        return dict(res=res, nu_i=nui, nu_o=nuo, status=st)

    def info(self, inst: int = 0) -> dict:
        out = (ctypes.c_int64 * 4)()
        _check(self._lib.lbm_axi_info(self._h, int(inst), out))
        return dict(t=out[0], t_check=out[1], status=RUN_STATE[out[2]], device_bytes=out[3])

    def derived(self, inst: int = 0) -> dict:
        """derived(cfg) of one instance's problem."""
        return derived(self.cfgs[inst])

    def set_tiles(self, kz: int, blocks_per_cu: int = 0):
        """Launch shape of the step kernel: nodes per thread along z and a cap
        on resident blocks per compute unit (0: none).  Results do not change."""
        _check(self._lib.lbm_axi_set_tiles(self._h, int(kz), int(blocks_per_cu)))

    def set_wall_lanes(self, mode: int = -1) -> bool:
        """Radial wall nodes computed by their own lanes (1) or by their owners
        after the owner's update (0); -1 restores the default chosen from the
        instances.  Returns the setting in force.  The variants agree up to
        FP32 rounding of the wall populations."""
        on = ctypes.c_int32(0)
        _check(self._lib.lbm_axi_set_wall_lanes(self._h, int(mode), ctypes.byref(on)))
        return bool(on.value)

    def set_storage(self, storage: str, storage_shift: int = 0):
        """Convert the populations to another storage type ("fp32", "fp16",
        "bf16") in place, keeping the state (precision handoff)."""
        code = STORAGE[storage] if isinstance(storage, str) else int(storage)
        _check(self._lib.lbm_axi_set_storage(self._h, code, int(storage_shift)))
        self.storage = storage

    def set_graph(self, steps: int):
        """Steps per captured step graph (even, 0 disables)."""
        _check(self._lib.lbm_axi_set_graph(self._h, int(steps)))

    def compact(self) -> int:
        """Drop finished instances from the step launch; returns the number running."""
        n = ctypes.c_int32()
        _check(self._lib.lbm_axi_compact(self._h, ctypes.byref(n)))
        return n.value

    def autotune(self, trial_steps: int = 20) -> dict:
        """Time every candidate launch shape on real steps and keep the fastest."""
        kz, bpc, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(self._lib.lbm_axi_autotune(self._h, int(trial_steps), ctypes.byref(kz),
                                          ctypes.byref(bpc), ctypes.byref(ms)))
        return dict(kz=kz.value, blocks_per_cu=bpc.value, ms=ms.value)

    def pattern_bandwidth(self, reps: int = 20) -> dict:
        """Streaming ceiling of the step's access pattern on this handle's arrays
        (GB/s of the even-step and odd-step patterns without arithmetic, of a
        plain read+write stream, and the algorithmic bytes of one step launch)."""
        out = (ctypes.c_double * 4)()
        _check(self._lib.lbm_axi_pattern_bandwidth(self._h, int(reps), out))
        return dict(even_gbs=out[0], odd_gbs=out[1], stream_gbs=out[2], bytes_per_launch=out[3])

    def lane_bandwidth(self, reps: int = 20) -> dict:
        """GB/s of an in-place stream over this handle's population arrays with
        lanes of 2, 4, 8 and 16 bytes (the state is left unchanged)."""
        out = (ctypes.c_double * 4)()
        _check(self._lib.lbm_axi_lane_bandwidth(self._h, int(reps), out))
        return {2: out[0], 4: out[1], 8: out[2], 16: out[3]}

    def set_timing(self, on: bool):
        _check(self._lib.lbm_axi_set_timing(self._h, 1 if on else 0))

    def kernel_time(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(self._lib.lbm_axi_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value
