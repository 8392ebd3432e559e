"""ctypes binding of the C ABI in ``include/lbm.h`` (same names, argument marshalling only).

Every step of the time-step path runs in the gfx950 kernels of ``liblbm.so``; PyTorch
only supplies the device memory (an arena tensor) and the HIP stream.  There is no CPU
path: if the library is missing or no gfx950 GPU is present, the calls fail loudly.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EUNSTABLE = 0, -1, -2, -3, -4, -5
STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE", -4: "LBM_ESTATE",
          -5: "LBM_EUNSTABLE"}
PRECISION = {"fp64": 0, "fp32": 1, "fp16s": 2}
SIDE = {"hot": 0, "cold": 1, "adiabatic": 2, "periodic": 3,
        "nee_hot": 4, "nee_cold": 5, "nee_adiabatic": 6, "nee_robin": 7}

# every symbol include/lbm.h declares
EXPORTS = (
    "lbm_params_default", "lbm_footprint_bytes", "lbm_create", "lbm_set_fields", "lbm_step",
    "lbm_observables", "lbm_observables_static", "lbm_get_fields", "lbm_get_derived", "lbm_derive",
    "lbm_state_bytes", "lbm_get_state",
    "lbm_set_state",
    "lbm_set_tile", "lbm_get_tile", "lbm_set_cache_policy", "lbm_get_cache_policy", "lbm_set_strip_width",
    "lbm_get_strip_width", "lbm_set_tile_rows", "lbm_get_tile_rows", "lbm_set_steps_per_launch",
    "lbm_get_steps_per_launch", "lbm_set_graph_chunk",
    "lbm_autotune", "lbm_last_error", "lbm_destroy",
    "lbm_batch_create", "lbm_batch_attach", "lbm_batch_detach", "lbm_batch_step", "lbm_batch_autotune",
    "lbm_batch_set_tile", "lbm_batch_size", "lbm_batch_destroy",
)
PRECISION_NAMES = ("fp64", "fp32", "fp16s")
BATCH_CLASSES = ("<=64", "<=128", "<=256", ">256")


class LbmError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("model", ctypes.c_int32), ("side", ctypes.c_int32 * 4),
        ("Ra", ctypes.c_double), ("Pr", ctypes.c_double), ("Le", ctypes.c_double),
        ("Da", ctypes.c_double), ("N", ctypes.c_double),
        ("J", ctypes.c_double), ("sigma", ctypes.c_double), ("phi", ctypes.c_double),
        ("Ma", ctypes.c_double), ("varpi", ctypes.c_double), ("rho0", ctypes.c_double),
        ("s_rho", ctypes.c_double), ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double),
        ("s_j", ctypes.c_double), ("s_q", ctypes.c_double),
        ("zeta0", ctypes.c_double), ("zeta_e", ctypes.c_double), ("zeta_eps", ctypes.c_double),
        ("eta0", ctypes.c_double), ("eta_e", ctypes.c_double), ("eta_eps", ctypes.c_double),
        ("Th", ctypes.c_double), ("Tl", ctypes.c_double), ("Ch", ctypes.c_double), ("Cl", ctypes.c_double),
        ("Fphi", ctypes.c_double), ("g_ext", ctypes.c_double * 2), ("wall_u", ctypes.c_double * 4),
        ("direct", ctypes.c_int32),
        ("nu", ctypes.c_double), ("alpha_e", ctypes.c_double), ("D_e", ctypes.c_double),
        ("K", ctypes.c_double), ("gbT", ctypes.c_double), ("gbC", ctypes.c_double),
        ("Bi_T", ctypes.c_double), ("Bi_C", ctypes.c_double),
        ("Re", ctypes.c_double), ("Gr", ctypes.c_double), ("U0", ctypes.c_double),
        ("stream", ctypes.c_void_p), ("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_uint64),
    ]


class Obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("Nu", ctypes.c_double * 4), ("Sh", ctypes.c_double * 4),
                ("mass", ctypes.c_double), ("heat", ctypes.c_double), ("solute", ctypes.c_double),
                ("max_ux", ctypes.c_double), ("max_uy", ctypes.c_double),
                ("r_u", ctypes.c_double), ("r_T", ctypes.c_double), ("r_C", ctypes.c_double),
                ("nonfinite", ctypes.c_int32)]


class Derived(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "L", "U", "nu", "nu_e", "alpha_e", "D_e", "s_v", "zeta_a", "eta_D", "varpi", "csT2",
        "gbT", "gbC", "T0", "C0", "dT", "dC", "K_mean", "phi_min", "fp16_scale")]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_VP = ctypes.c_void_p


def lib():
    """Load ``liblbm.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.lbm_params_default.argtypes = [ctypes.POINTER(Params)]
        L.lbm_params_default.restype = None
        L.lbm_footprint_bytes.argtypes = [ctypes.POINTER(Params)]
        L.lbm_footprint_bytes.restype = ctypes.c_uint64
        L.lbm_create.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(_VP)]
        L.lbm_set_fields.argtypes = [_VP, _D, _D, _D, _D, _D]
        L.lbm_step.argtypes = [_VP, ctypes.c_int64]
        L.lbm_observables.argtypes = [_VP, ctypes.POINTER(Obs), _D]
        L.lbm_observables_static.argtypes = [_VP, ctypes.POINTER(Obs), _D]
        L.lbm_get_fields.argtypes = [_VP, _D]
        L.lbm_get_derived.argtypes = [_VP, ctypes.POINTER(Derived)]
        L.lbm_derive.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Derived)]
        L.lbm_state_bytes.argtypes = [_VP]
        L.lbm_state_bytes.restype = ctypes.c_uint64
        L.lbm_get_state.argtypes = [_VP, _VP, ctypes.c_uint64]
        L.lbm_set_state.argtypes = [_VP, _VP, ctypes.c_uint64]
        L.lbm_set_cache_policy.argtypes = [_VP, ctypes.c_int32]
        L.lbm_set_cache_policy.restype = ctypes.c_int
        L.lbm_get_cache_policy.argtypes = [_VP]
        L.lbm_get_cache_policy.restype = ctypes.c_int32
        L.lbm_set_strip_width.argtypes = [_VP, ctypes.c_int32]
        L.lbm_set_strip_width.restype = ctypes.c_int
        L.lbm_get_strip_width.argtypes = [_VP]
        L.lbm_get_strip_width.restype = ctypes.c_int32
        L.lbm_set_tile_rows.argtypes = [_VP, ctypes.c_int32]
        L.lbm_set_tile_rows.restype = ctypes.c_int
        L.lbm_get_tile_rows.argtypes = [_VP]
        L.lbm_get_tile_rows.restype = ctypes.c_int32
        L.lbm_set_steps_per_launch.argtypes = [_VP, ctypes.c_int32]
        L.lbm_set_steps_per_launch.restype = ctypes.c_int
        L.lbm_get_steps_per_launch.argtypes = [_VP]
        L.lbm_get_steps_per_launch.restype = ctypes.c_int32
        L.lbm_set_tile.argtypes = [_VP, ctypes.c_int32, ctypes.c_int32]
        L.lbm_set_graph_chunk.argtypes = [_VP, ctypes.c_int32]
        L.lbm_get_tile.argtypes = [_VP, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.lbm_autotune.argtypes = [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
        L.lbm_last_error.argtypes = [_VP]
        L.lbm_last_error.restype = ctypes.c_char_p
        L.lbm_destroy.argtypes = [_VP]
        L.lbm_destroy.restype = None
        L.lbm_batch_create.argtypes = [ctypes.c_int32, ctypes.c_int32, _VP, ctypes.POINTER(_VP)]
        L.lbm_batch_attach.argtypes = [_VP, _VP]
        L.lbm_batch_detach.argtypes = [_VP, _VP]
        L.lbm_batch_step.argtypes = [_VP, ctypes.c_int64]
        L.lbm_batch_autotune.argtypes = [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32)]
        L.lbm_batch_set_tile.argtypes = [_VP] + [ctypes.c_int32] * 4
        L.lbm_batch_size.argtypes = [_VP]
        L.lbm_batch_size.restype = ctypes.c_int32
        L.lbm_batch_destroy.argtypes = [_VP]
        L.lbm_batch_destroy.restype = None
        _lib = L
    return _lib


def _check(rc, handle=None, what=""):
    if rc != OK:
        msg = lib().lbm_last_error(handle).decode() if handle else what
        raise LbmError(rc, f"{what}: {msg}" if what else msg)


def make_params(p: dict, precision: str = "fp32") -> Params:
    """lbm_params from a problem-statement dictionary (missing keys keep the defaults of
    lbm_params_default)."""
    s = Params()
    lib().lbm_params_default(ctypes.byref(s))
    s.precision = PRECISION[precision]
    for k, v in p.items():
        if k == "precision":
            continue
        if k == "sides":
            s.side = (ctypes.c_int32 * 4)(*[SIDE[x] if isinstance(x, str) else int(x) for x in v])
        elif k == "g_ext":
            s.g_ext = (ctypes.c_double * 2)(*v)
        elif k == "wall_u":
            s.wall_u = (ctypes.c_double * 4)(*v)
        elif k in dict(Params._fields_):
            setattr(s, k, v)
        else:
            raise KeyError(f"unknown parameter {k!r}")
    return s


def node_walls(params: dict) -> bool:
    """True when a side of the problem is a wall through the boundary nodes (side kinds 4-7,
    by name or number)."""
    for k in params.get("sides", ()):
        if (isinstance(k, str) and k.startswith("nee_")) or (not isinstance(k, str) and int(k) >= 4):
            return True
    return False


def derive(p: dict, precision: str = "fp32") -> dict:
    """lbm_derive: the lattice values of a problem statement for its uniform porosity, computed
    on the host (no device needed)."""
    s = make_params(p, precision)
    d = Derived()
    _check(lib().lbm_derive(ctypes.byref(s), ctypes.byref(d)), None, "lbm_derive")
    return {n: getattr(d, n) for n, _ in Derived._fields_}


def footprint_bytes(p: dict, precision: str = "fp32") -> int:
    s = make_params(p, precision)
    return int(lib().lbm_footprint_bytes(ctypes.byref(s)))


def _host(a, shape):
    if a is None:
        return None
    return np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), shape))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_D)


class Solver:
    """One cavity on the GPU.  ``precision`` is 'fp64', 'fp32' or 'fp16s'.  Device memory
    comes from a torch arena tensor on ``device`` and work runs on torch's current stream of
    that device (or ``stream``, a torch.cuda.Stream).  ``tile``: (tile_x, tile_y), or "auto"
    for the cached autotuned shape of this lattice class (timed once per class)."""

    def __init__(self, params: dict, phi=None, T=None, C=None, ux=None, uy=None, precision="fp32",
                 device=None, stream=None, tile=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the lattice Boltzmann library runs only on a gfx950 GPU")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.precision = precision
        self._batch = None          # the Batch this solver is attached to
        self.p = dict(params)
        self.nx, self.ny = int(params.get("nx", 64)), int(params.get("ny", 64))
        self._s = make_params(params, precision)
        with torch.cuda.device(self.device):
            self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            nbytes = int(lib().lbm_footprint_bytes(ctypes.byref(self._s)))
            self._arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self._s.arena = self._arena.data_ptr()
            self._s.arena_bytes = nbytes
            self._s.stream = self._stream.cuda_stream
            h = _VP()
            _check(lib().lbm_create(ctypes.byref(self._s), ctypes.byref(h)), None, "lbm_create")
            self._h = h
            shape = (self.ny, self.nx)
            arrs = [_host(a, shape) for a in (phi, T, C, ux, uy)]
            _check(lib().lbm_set_fields(self._h, *[_ptr(a) for a in arrs]), self._h, "lbm_set_fields")
            if tile == "auto":
                from . import autotune
                autotune.tune(self, torch.cuda.get_device_name(self.device), phi is not None,
                              node_walls=node_walls(params))
            elif tile is not None:
                self.set_tile(*tile)

    @property
    def handle(self):
        return self._h

    def step(self, n: int = 1):
        _check(lib().lbm_step(self._h, int(n)), self._h, "lbm_step")

    def observables(self, fields: bool = False, static: bool = False):
        """lbm_observables, or with ``static`` lbm_observables_static (no device allocation;
        the library's fixed scratch)."""
        o = Obs()
        buf = np.empty((5, self.ny, self.nx)) if fields else None
        fn = lib().lbm_observables_static if static else lib().lbm_observables
        rc = fn(self._h, ctypes.byref(o), _ptr(buf))
        if rc not in (OK, EUNSTABLE):
            _check(rc, self._h, "lbm_observables_static" if static else "lbm_observables")
        ob = dict(step=o.step, Nu=list(o.Nu), Sh=list(o.Sh), mass=o.mass, heat=o.heat, solute=o.solute,
                  max_ux=o.max_ux, max_uy=o.max_uy, r_u=o.r_u, r_T=o.r_T, r_C=o.r_C,
                  nonfinite=bool(o.nonfinite), status=rc)
        if fields:
            ob["fields"] = dict(zip(("rho", "ux", "uy", "T", "C"), buf))
        return ob

    def fields(self):
        """FP64 fields rho, ux, uy, T, C of the current level, each (ny, nx)."""
        buf = np.empty((5, self.ny, self.nx))
        _check(lib().lbm_get_fields(self._h, _ptr(buf)), self._h, "lbm_get_fields")
        return dict(zip(("rho", "ux", "uy", "T", "C"), buf))

    def derived(self) -> dict:
        d = Derived()
        _check(lib().lbm_get_derived(self._h, ctypes.byref(d)), self._h, "lbm_get_derived")
        return {n: getattr(d, n) for n, _ in Derived._fields_}

    def get_state(self) -> bytes:
        n = int(lib().lbm_state_bytes(self._h))
        buf = ctypes.create_string_buffer(n)
        _check(lib().lbm_get_state(self._h, buf, n), self._h, "lbm_get_state")
        return buf.raw

    def set_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().lbm_set_state(self._h, buf, len(blob)), self._h, "lbm_set_state")

    def set_tile(self, tx: int, ty: int):
        _check(lib().lbm_set_tile(self._h, int(tx), int(ty)), self._h, "lbm_set_tile")

    def set_graph_chunk(self, chunk: int):
        _check(lib().lbm_set_graph_chunk(self._h, int(chunk)), self._h, "lbm_set_graph_chunk")

    def set_cache_policy(self, policy: int):
        """0 tuned, 1 streaming, 2 resident, -1 the default rule (see include/lbm.h)."""
        _check(lib().lbm_set_cache_policy(self._h, int(policy)), self._h, "lbm_set_cache_policy")

    def get_cache_policy(self) -> int:
        return int(lib().lbm_get_cache_policy(self._h))

    def set_strip_width(self, tiles: int):
        """Tile order of the multi-step launches: 0 row by row, k >= 1 vertical strips of k
        tiles, -1 the default rule (see include/lbm.h)."""
        _check(lib().lbm_set_strip_width(self._h, int(tiles)), self._h, "lbm_set_strip_width")

    def get_strip_width(self) -> int:
        return int(lib().lbm_get_strip_width(self._h))

    def set_tile_rows(self, rows: int):
        """Rows of the FP32 three-step and FP16 two-step tile: 8, 12 or 0 for the default rule
        (see include/lbm.h)."""
        _check(lib().lbm_set_tile_rows(self._h, int(rows)), self._h, "lbm_set_tile_rows")

    def get_tile_rows(self) -> int:
        return int(lib().lbm_get_tile_rows(self._h))

    def set_steps_per_launch(self, n: int):
        """1, 2 (two-step LDS kernel), 3 (three-step LDS kernel) or 0 for the default (see
        include/lbm.h)."""
        _check(lib().lbm_set_steps_per_launch(self._h, int(n)), self._h, "lbm_set_steps_per_launch")

    def get_steps_per_launch(self) -> int:
        return int(lib().lbm_get_steps_per_launch(self._h))

    def get_tile(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().lbm_get_tile(self._h, ctypes.byref(a), ctypes.byref(b)), self._h, "lbm_get_tile")
        return a.value, b.value

    def autotune(self, steps: int = 20):
        a, b, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(lib().lbm_autotune(self._h, int(steps), ctypes.byref(a), ctypes.byref(b), ctypes.byref(ms)),
               self._h, "lbm_autotune")
        return (a.value, b.value), ms.value

    def close(self):
        if getattr(self, "_h", None):
            b = getattr(self, "_batch", None)
            if b is not None and self in b.members:
                b.members.remove(self)     # lbm_destroy detaches it from the batch
            self._batch = None
            lib().lbm_destroy(self._h)
            self._h = None
            self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Batched stepping of many Solvers with one launch per precision per time step,
    replayed from a captured HIP graph of ``chunk`` steps."""

    def __init__(self, max_cavities: int, chunk: int = 100, stream=None, device=None):
        import torch
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = _VP()
        _check(lib().lbm_batch_create(int(max_cavities), int(chunk), self._stream.cuda_stream, ctypes.byref(h)),
               None, "lbm_batch_create")
        self._h = h
        self.members = []

    def attach(self, s: Solver):
        _check(lib().lbm_batch_attach(self._h, s.handle), s.handle, "lbm_batch_attach")
        self.members.append(s)
        s._batch = self

    def detach(self, s: Solver):
        _check(lib().lbm_batch_detach(self._h, s.handle), s.handle, "lbm_batch_detach")
        self.members.remove(s)
        s._batch = None

    def step(self, n: int):
        _check(lib().lbm_batch_step(self._h, int(n)), None, "lbm_batch_step")

    def autotune(self, steps: int = 20) -> dict:
        """lbm_batch_autotune: the tile shape index and cache policy chosen for each precision
        and size class present, as {(precision, class): (shape, policy)}."""
        shapes = (ctypes.c_int32 * 12)(*([-1] * 12))
        pols = (ctypes.c_int32 * 12)(*([-1] * 12))
        _check(lib().lbm_batch_autotune(self._h, int(steps), shapes, pols), None, "lbm_batch_autotune")
        out = {}
        for i in range(12):
            if shapes[i] >= 0:
                out[(PRECISION_NAMES[i // 4], BATCH_CLASSES[i % 4])] = (int(shapes[i]), int(pols[i]))
        return out

    def set_tile(self, precision: str, size_class: int, shape: int, policy: int = -1):
        """lbm_batch_set_tile: the launch choice of one precision and size class (shape 0-2:
        two-step tiles; 3: three steps per launch, FP32 and FP64, with a chunk that is a
        multiple of 12)."""
        _check(lib().lbm_batch_set_tile(self._h, PRECISION[precision], int(size_class), int(shape), int(policy)),
               None, "lbm_batch_set_tile")

    def __len__(self):
        return int(lib().lbm_batch_size(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_batch_destroy(self._h)
            self._h = None
            for s in self.members:
                s._batch = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
