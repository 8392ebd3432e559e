"""C-ABI checks that need no GPU: the library loads, exports every function the header
declares, and rejects invalid parameters before touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1708_07525_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_symbol():
    lbm.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", lbm.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(lbm_\w+)", out))
    declared = set(declared_functions())
    assert declared, "no declarations parsed"
    assert declared <= exported, declared - exported
    assert declared == set(lbm.EXPORTS)
    # nothing else leaks out of the library
    assert exported == declared, exported - declared


def test_param_struct_matches_header_defaults():
    p = lbm.make_params({})
    assert (p.nx, p.ny, p.precision, p.model) == (64, 64, 1, 0)
    assert list(p.side) == [0, 1, 2, 2]
    assert (p.s_e, p.s_eps, p.s_q, p.s_j, p.s_rho) == (1.1, 1.1, 1.2, 1.0, 1.0)
    assert (p.zeta0, p.zeta_e, p.zeta_eps, p.eta0, p.eta_e, p.eta_eps) == (1.0, 1.5, 1.5, 1.0, 1.5, 1.5)
    assert (p.rho0, p.J, p.sigma, p.Ma, p.varpi, p.Fphi) == (1.0, 1.0, 1.0, 0.1, 0.0, -1.0)
    # ctypes layout agrees with the C struct: footprint computation reads nx/ny/precision
    assert lbm.footprint_bytes({"nx": 64, "ny": 64}, "fp32") > 64 * 64 * 38 * 4


def test_footprint_scales_with_precision():
    f64 = lbm.footprint_bytes({"nx": 1024, "ny": 1024}, "fp64")
    f32 = lbm.footprint_bytes({"nx": 1024, "ny": 1024}, "fp32")
    f16 = lbm.footprint_bytes({"nx": 1024, "ny": 1024}, "fp16s")
    n = 1024 * 1024
    # populations in two buffers; fields in two buffers, porosity, residual snapshot (13 planes)
    assert 2 * 19 * 8 * n < f64 < 1.1 * (2 * 19 * 8 + 13 * 8) * n
    assert 2 * 19 * 4 * n < f32 < 1.1 * (2 * 19 * 4 + 13 * 4) * n
    assert 2 * 19 * 2 * n < f16 < 1.1 * (2 * 19 * 2 + 13 * 4) * n
    assert lbm.footprint_bytes({"nx": 2, "ny": 64}) == 0


@pytest.mark.parametrize("bad", [
    {"nx": 2}, {"ny": 1}, {"phi": 0.0}, {"phi": 1.5}, {"s_e": 2.0}, {"zeta_e": 0.0}, {"Ra": -1.0},
    {"Pr": 0.0}, {"Le": 0.0}, {"Da": 0.0}, {"Th": 0.0, "Tl": 1.0}, {"model": 3}, {"varpi": 1.2},
    {"sides": ("periodic", "cold", "adiabatic", "adiabatic")}, {"sides": (0, 1, 2, 7)}, {"sides": (0, 1, 2, 8)},
    {"sides": ("nee_hot", "cold", "adiabatic", "adiabatic")},
    {"sides": ("nee_hot", "nee_robin", "nee_adiabatic", "nee_adiabatic"), "Bi_T": -1.0},
    {"sides": ("nee_hot", "nee_robin", "nee_adiabatic", "nee_adiabatic"), "Bi_C": -0.5},
    {"nx": 4, "sides": ("nee_hot", "nee_cold", "nee_adiabatic", "nee_adiabatic")},
    {"direct": 1, "nu": 0.0, "alpha_e": 0.1, "D_e": 0.1, "K": 1.0},
    {"direct": 2, "Re": 0.0, "Gr": 100.0, "U0": 0.1}, {"direct": 2, "Re": 100.0, "Gr": -1.0, "U0": 0.1},
    {"direct": 2, "Re": 100.0, "Gr": 100.0, "U0": 0.0}, {"direct": 3},
    # population planes beyond the 4 GiB range of one buffer resource
    {"nx": 8192, "ny": 8192, "precision": "fp32"}, {"nx": 6144, "ny": 6144, "precision": "fp64"},
    {"nx": 11264, "ny": 11264, "precision": "fp16s"},
])
def test_create_rejects_invalid_parameters(bad):
    bad = dict(bad)
    p = lbm.make_params(bad, bad.pop("precision", "fp32"))
    h = ctypes.c_void_p()
    rc = lbm.lib().lbm_create(ctypes.byref(p), ctypes.byref(h))
    assert rc == lbm.EINVAL
    assert not h.value


def test_null_arguments():
    L = lbm.lib()
    assert L.lbm_create(None, None) == lbm.EINVAL
    assert L.lbm_step(None, 1) == lbm.EINVAL
    assert L.lbm_observables(None, None, None) == lbm.EINVAL
    assert L.lbm_set_fields(None, None, None, None, None, None) == lbm.EINVAL
    L.lbm_destroy(None)
    assert L.lbm_last_error(None) == b"no context"
    assert L.lbm_batch_step(None, 1) == lbm.EINVAL
    assert L.lbm_batch_size(None) == 0
    L.lbm_batch_destroy(None)
    assert L.lbm_batch_create(0, 2, None, ctypes.byref(ctypes.c_void_p())) == lbm.EINVAL
    assert L.lbm_batch_create(4, 3, None, ctypes.byref(ctypes.c_void_p())) == lbm.EINVAL


def test_solver_refuses_to_run_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        lbm.Solver({"nx": 16, "ny": 16})


# the largest lattices whose 19 population planes (rows padded to 64 nodes, planes to 1024
# elements plus 256) fit in 4 GiB, and the next row up
LARGEST = [("fp32", 7500, 7482), ("fp64", 5300, 5319), ("fp16s", 10600, 10638)]


@pytest.mark.parametrize("prec,nx,ny", LARGEST)
def test_largest_lattice_is_accepted_and_the_next_row_refused(prec, nx, ny):
    es = {"fp32": 4, "fp64": 8, "fp16s": 2}[prec]
    pitch = -(-nx // 64) * 64

    def planes_bytes(rows):
        return 19 * (-(-pitch * rows // 1024) * 1024 + 256) * es

    assert planes_bytes(ny) < 2 ** 32 <= planes_bytes(ny + 1)
    for rows, ok in ((ny, True), (ny + 1, False)):
        p = lbm.make_params({"nx": nx, "ny": rows}, prec)
        h = ctypes.c_void_p()
        rc = lbm.lib().lbm_create(ctypes.byref(p), ctypes.byref(h))
        # without a GPU an accepted lattice fails later, at the device (never LBM_EINVAL)
        assert (rc != lbm.EINVAL) if ok else (rc == lbm.EINVAL)
        if h.value:
            lbm.lib().lbm_destroy(h)


def test_derived_values_of_the_natural_convection_mapping():
    """lbm_derive (host only) on the 64x64 porous cavity: the hand values of section 4.1 and
    Eq. (29) (the same numbers pin the oracle's own mapping)."""
    d = lbm.derive({})
    hand = dict(U=0.0577350, nu=0.0369504, s_v=1.637060, zeta_a=1.460383, eta_D=1.688117, gbT=5.208333e-5,
                gbC=5.208333e-5, K_mean=40.96, varpi=0.4, L=64.0)
    for k, v in hand.items():
        assert d[k] == pytest.approx(v, rel=2e-6), k


def test_derived_values_of_the_lid_driven_mapping():
    """Section 4.3 (Table 4 case, 128^2, Re = Gr = 100, U0 = 0.1, Da = 0.1, N = -500): nu =
    U0 L/Re = 0.128, 1/s_v = 1/2 + J L U0/(c_s^2 Re) = 0.884, g beta_T dT = Gr nu^2/L^3 =
    7.8125e-7, K = 1638.4, zeta_alpha = eta_D = 1/1.14; with walls through the nodes L = 128
    on 129 nodes gives the same values."""
    base = dict(sides=("adiabatic", "adiabatic", "cold", "hot"), direct=2, Re=100.0, Gr=100.0, U0=0.1, Pr=1.0,
                Le=1.0, Da=0.1, N=-500.0, phi=0.95, wall_u=(0.0, 0.0, 0.0, 0.1))
    hand = dict(nu=0.128, s_v=1 / 0.884, gbT=7.8125e-7, gbC=-500 * 7.8125e-7, K_mean=1638.4, zeta_a=1 / 1.14,
                eta_D=1 / 1.14, U=0.1, L=128.0)
    for p in (dict(base, nx=128, ny=128),
              dict(base, nx=129, ny=129, sides=("nee_adiabatic", "nee_adiabatic", "nee_cold", "nee_hot"))):
        d = lbm.derive(p, "fp64")
        for k, v in hand.items():
            assert d[k] == pytest.approx(v, rel=1e-12), (p["nx"], k)
    with pytest.raises(lbm.LbmError):
        lbm.derive(dict(base, nx=128, ny=128, Re=-1.0))
