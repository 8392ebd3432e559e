"""FP64 CPU oracle of the Liu & He MRT lattice Boltzmann model (arXiv 1708.07525).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  It shares no code with the GPU
library: the C source ``orc.c`` writes every step of the method out from the paper
(Eqs. 5-29, section 4.1) with explicit matrices, in double precision.

Parameters are plain dictionaries with the keys of ``DEFAULTS``; fields are numpy
float64 arrays of shape (ny, nx), x fastest.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")

SIDE = {"hot": 0, "cold": 1, "adiabatic": 2, "periodic": 3,
        "nee_hot": 4, "nee_cold": 5, "nee_adiabatic": 6, "nee_robin": 7}
MUTATION = {"none": 0, "no_source": 1, "no_half_force": 2, "rho_in_meq": 3, "buoy_sign": 4,
            "model_a_diff": 5, "no_forch": 6, "wall_const": 7, "ergun_exp": 8, "wall_vel": 9,
            "model_a_map": 10, "nee_wall_vel": 11}

# Section 4 constants: rho0 = J = sigma = 1, varpi = 2/5 (here: automatic, see varpi),
# s_rho = s_j = 1, s_e = s_eps = 1.1, s_q = 1.2, zeta0 = eta0 = 1, zeta_e,eps = eta_e,eps = 1.5.
DEFAULTS = dict(
    nx=64, ny=64, model=0, mutation="none",
    sides=("hot", "cold", "adiabatic", "adiabatic"),
    Ra=1e4, Pr=1.0, Le=2.0, Da=1e-2, N=1.0,
    J=1.0, sigma=1.0, phi=0.6,
    Ma=0.1, varpi=0.0, rho0=1.0,
    s_rho=1.0, s_e=1.1, s_eps=1.1, s_j=1.0, s_q=1.2,
    zeta0=1.0, zeta_e=1.5, zeta_eps=1.5, eta0=1.0, eta_e=1.5, eta_eps=1.5,
    Th=1.0, Tl=0.0, Ch=1.0, Cl=0.0,
    Fphi=-1.0, g_ext=(0.0, 0.0), wall_u=(0.0, 0.0, 0.0, 0.0),
    direct=0, nu=0.0, alpha_e=0.0, D_e=0.0, K=0.0, gbT=0.0, gbC=0.0, Bi_T=0.0, Bi_C=0.0,
    Re=0.0, Gr=0.0, U0=0.0, nee_link=0,
)


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("model", ctypes.c_int32),
        ("mutation", ctypes.c_int32), ("side", ctypes.c_int32 * 4),
        ("Ra", ctypes.c_double), ("Pr", ctypes.c_double), ("Le", ctypes.c_double),
        ("Da", ctypes.c_double), ("N", ctypes.c_double),
        ("J", ctypes.c_double), ("sigma", ctypes.c_double), ("phi", ctypes.c_double),
        ("Ma", ctypes.c_double), ("varpi", ctypes.c_double), ("rho0", ctypes.c_double),
        ("s_rho", ctypes.c_double), ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double),
        ("s_j", ctypes.c_double), ("s_q", ctypes.c_double),
        ("zeta0", ctypes.c_double), ("zeta_e", ctypes.c_double), ("zeta_eps", ctypes.c_double),
        ("eta0", ctypes.c_double), ("eta_e", ctypes.c_double), ("eta_eps", ctypes.c_double),
        ("Th", ctypes.c_double), ("Tl", ctypes.c_double), ("Ch", ctypes.c_double),
        ("Cl", ctypes.c_double), ("Fphi", ctypes.c_double), ("g_ext", ctypes.c_double * 2),
        ("wall_u", ctypes.c_double * 4), ("direct", ctypes.c_int32),
        ("nu", ctypes.c_double), ("alpha_e", ctypes.c_double), ("D_e", ctypes.c_double),
        ("K", ctypes.c_double), ("gbT", ctypes.c_double), ("gbC", ctypes.c_double),
        ("Bi_T", ctypes.c_double), ("Bi_C", ctypes.c_double),
        ("Re", ctypes.c_double), ("Gr", ctypes.c_double), ("U0", ctypes.c_double),
        ("nee_link", ctypes.c_int32),
    ]


class _Derived(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "L", "U", "nu", "nu_e", "alpha_e", "D_e", "s_v", "zeta_a", "eta_D", "varpi", "csT2",
        "gbT", "gbC", "T0", "C0", "dT", "dC", "K_mean", "phi_min")]


class _Obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("Nu", ctypes.c_double * 4), ("Sh", ctypes.c_double * 4),
                ("mass", ctypes.c_double), ("heat", ctypes.c_double), ("solute", ctypes.c_double),
                ("max_ux", ctypes.c_double), ("max_uy", ctypes.c_double),
                ("r_u", ctypes.c_double), ("r_T", ctypes.c_double), ("r_C", ctypes.c_double),
                ("nonfinite", ctypes.c_int32)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.POINTER(_Params)]
        L.orc_set_fields.argtypes = [ctypes.c_void_p] + [_D] * 5
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.orc_macro.argtypes = [ctypes.c_void_p] + [_D] * 5
        L.orc_observables.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Obs)]
        L.orc_derived_values.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Derived)]
        L.orc_get_populations.argtypes = [ctypes.c_void_p, _D, _D, _D]
        L.orc_set_populations.argtypes = [ctypes.c_void_p, _D, _D, _D]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_matrices.argtypes = [_D] * 4
        L.orc_meq.argtypes = [ctypes.c_double] * 5 + [_D]
        L.orc_feq.argtypes = [ctypes.c_double] * 5 + [_D]
        L.orc_force_moments.argtypes = [ctypes.c_double] * 6 + [_D]
        L.orc_geq.argtypes = [ctypes.c_double] * 5 + [ctypes.c_int, _D]
        L.orc_ngeq.argtypes = [ctypes.c_double] * 5 + [ctypes.c_int, _D]
        L.orc_source5.argtypes = [ctypes.c_double] * 3 + [_D]
        L.orc_velocity.argtypes = [ctypes.c_double] * 4 + [_D, _D]
        L.orc_node_coeffs.argtypes = [ctypes.c_void_p, ctypes.c_long, _D]
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_D)


def _f64(a, shape):
    if a is None:
        return None
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), shape))
    return a


def make_params(**kw) -> dict:
    p = dict(DEFAULTS)
    for k, v in kw.items():
        if k not in p:
            raise KeyError(f"unknown parameter {k!r}")
        p[k] = v
    return p


def _to_struct(p: dict) -> _Params:
    s = _Params()
    for name, _t in _Params._fields_:
        if name == "side":
            s.side = (ctypes.c_int32 * 4)(*[SIDE[x] if isinstance(x, str) else int(x) for x in p["sides"]])
        elif name == "mutation":
            m = p["mutation"]
            s.mutation = MUTATION[m] if isinstance(m, str) else int(m)
        elif name == "g_ext":
            s.g_ext = (ctypes.c_double * 2)(*p["g_ext"])
        elif name == "wall_u":
            s.wall_u = (ctypes.c_double * 4)(*p["wall_u"])
        else:
            setattr(s, name, p[name])
    return s


class Oracle:
    """One cavity advanced by the FP64 oracle.  ``fields()`` returns the macroscopic
    fields (rho, ux, uy, T, C) of the current time level, each (ny, nx)."""

    def __init__(self, params: dict, phi=None, T=None, C=None, ux=None, uy=None):
        self.p = make_params(**params)
        self.nx, self.ny = int(self.p["nx"]), int(self.p["ny"])
        self._s = _to_struct(self.p)
        self._h = lib().orc_create(ctypes.byref(self._s))
        if not self._h:
            raise ValueError("orc_create rejected the parameters")
        shape = (self.ny, self.nx)
        arrs = [_f64(a, shape) for a in (phi, T, C, ux, uy)]
        rc = lib().orc_set_fields(self._h, *[_ptr(a) for a in arrs])
        if rc != 0:
            raise ValueError("orc_set_fields rejected the fields")

    def step(self, n: int = 1):
        if lib().orc_step(self._h, int(n)) != 0:
            raise RuntimeError("orc_step failed")

    def fields(self):
        shape = (self.ny, self.nx)
        out = [np.empty(shape) for _ in range(5)]
        lib().orc_macro(self._h, *[_ptr(a) for a in out])
        return dict(zip(("rho", "ux", "uy", "T", "C"), out))

    def observables(self) -> dict:
        o = _Obs()
        if lib().orc_observables(self._h, ctypes.byref(o)) != 0:
            raise RuntimeError("orc_observables failed")
        return dict(step=o.step, Nu=list(o.Nu), Sh=list(o.Sh), mass=o.mass, heat=o.heat,
                    solute=o.solute, max_ux=o.max_ux, max_uy=o.max_uy, r_u=o.r_u, r_T=o.r_T,
                    r_C=o.r_C, nonfinite=bool(o.nonfinite))

    def derived(self) -> dict:
        d = _Derived()
        lib().orc_derived_values(self._h, ctypes.byref(d))
        return {n: getattr(d, n) for n, _ in _Derived._fields_}

    def node_coeffs(self, x: int, y: int) -> dict:
        """Porous coefficients at node (x, y): K, F_phi (Eq. 7) and l0, l1 (Eq. 19)."""
        out = np.empty(4)
        if lib().orc_node_coeffs(self._h, int(y) * self.nx + int(x), _ptr(out)) != 0:
            raise ValueError("orc_node_coeffs failed")
        return dict(zip(("K", "Fphi", "l0", "l1"), out.tolist()))

    def populations(self):
        nn = self.nx * self.ny
        f, g, h = np.empty((9, self.ny, self.nx)), np.empty((5, self.ny, self.nx)), np.empty((5, self.ny, self.nx))
        lib().orc_get_populations(self._h, _ptr(f), _ptr(g), _ptr(h))
        assert f.size == 9 * nn
        return f, g, h

    def set_populations(self, f=None, g=None, h=None):
        f = _f64(f, (9, self.ny, self.nx))
        g = _f64(g, (5, self.ny, self.nx))
        h = _f64(h, (5, self.ny, self.nx))
        lib().orc_set_populations(self._h, _ptr(f), _ptr(g), _ptr(h))

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def matrices():
    M, Mi, N, Ni = np.empty((9, 9)), np.empty((9, 9)), np.empty((5, 5)), np.empty((5, 5))
    lib().orc_matrices(_ptr(M), _ptr(Mi), _ptr(N), _ptr(Ni))
    return M, Mi, N, Ni


def meq(rho, ux, uy, phi, rho0=1.0):
    out = np.empty(9)
    lib().orc_meq(rho, ux, uy, phi, rho0, _ptr(out))
    return out


def feq(rho, ux, uy, phi, rho0=1.0):
    out = np.empty(9)
    lib().orc_feq(rho, ux, uy, phi, rho0, _ptr(out))
    return out


def force_moments(ux, uy, Fx, Fy, phi, rho0=1.0):
    out = np.empty(9)
    lib().orc_force_moments(ux, uy, Fx, Fy, phi, rho0, _ptr(out))
    return out


def geq(T, ux, uy, cap, varpi, model=0):
    out = np.empty(5)
    lib().orc_geq(T, ux, uy, cap, varpi, model, _ptr(out))
    return out


def ngeq(T, ux, uy, cap, varpi, model=0):
    out = np.empty(5)
    lib().orc_ngeq(T, ux, uy, cap, varpi, model, _ptr(out))
    return out


def source5(ax, ay, varpi):
    out = np.empty(5)
    lib().orc_source5(ax, ay, varpi, _ptr(out))
    return out


def velocity(vx, vy, l0, l1):
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().orc_velocity(vx, vy, l0, l1, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """OpenMP threads for the following steps: n > 0 sets n, 0 restores the default."""
    lib().orc_set_threads(int(n))
