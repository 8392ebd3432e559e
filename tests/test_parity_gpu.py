"""Parity of the gfx950 path (through the C ABI) with the FP64 CPU oracle.

Field error e_X = max|X_gpu - X_oracle| / max|X_oracle| for X in T, C; for the velocity
components the denominator is the largest speed max|u_oracle| (a component that is still
near zero early in a run would otherwise turn round-off into a large ratio); rho is
compared as an absolute error.  Bars: FP64 storage 1e-10, FP32 storage 1e-5 (both after
the stated number of steps on the same seeded inputs); FP16 storage is reported and held
to the bound derived for binary16 deviations (see test_fp16s_error_bound).
"""
import numpy as np
import pytest

import workloads
from oracle import Oracle
from tests import pins

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}


def _state_diff(a: bytes, b: bytes):
    """None when two state blobs are bitwise equal, else a short description (pytest's own
    diff of two large byte strings takes minutes)."""
    if a == b:
        return None
    if len(a) != len(b):
        return f"sizes {len(a)} != {len(b)}"
    x, y = np.frombuffer(a, np.uint8), np.frombuffer(b, np.uint8)
    bad = np.nonzero(x != y)[0]
    return f"{bad.size} of {x.size} bytes differ, first at offset {bad[0]}"


def _solver():
    from paper_1708_07525_amd import Solver
    return Solver


def make_gpu(prec):
    def mk(params, **fields):
        return _solver()(params, precision=prec, **fields)
    return mk


def field_errors(F, R):
    e = {k: float(np.abs(F[k] - R[k]).max() / max(np.abs(R[k]).max(), 1e-300)) for k in ("T", "C")}
    speed = max(float(np.hypot(R["ux"], R["uy"]).max()), 1e-300)
    for k in ("ux", "uy"):
        e[k] = float(np.abs(F[k] - R[k]).max()) / speed
    e["rho"] = float(np.abs(F["rho"] - R["rho"]).max())
    return e


def run_pair(params, steps, prec, phi=None, T=None, C=None, ux=None, uy=None, tile=None):
    print(f"case nx={params.get('nx')} ny={params.get('ny')} prec={prec} steps={steps} tile={tile}", flush=True)
    ref = Oracle(params, phi=phi, T=T, C=C, ux=ux, uy=uy)
    gpu = _solver()(params, phi=phi, T=T, C=C, ux=ux, uy=uy, precision=prec, tile=tile)
    ref.step(steps)
    gpu.step(steps)
    return gpu, ref, field_errors(gpu.fields(), ref.fields())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_small_cavity(prec):
    case = workloads.small_cavity(seed=0)
    gpu, ref, e = run_pair(case["params"], 1000, prec, T=case["T"], C=case["C"])
    print(prec, e, flush=True)
    assert max(e.values()) <= TOL[prec], e


@pytest.mark.parametrize("prec,tile", [("fp64", (64, 4)), ("fp32", (256, 8)), ("fp32", (128, 2))])
def test_ragged_nonsquare(prec, tile):
    p = workloads.cavity_params(nx=96, ny=67, Ra=3e4, Da=5e-3, Le=3.0, N=-0.5, phi=0.7)
    T, C = workloads.noise_fields(96, 67, 11)
    _, _, e = run_pair(p, 500, prec, T=T, C=C, tile=tile)
    assert max(e.values()) <= TOL[prec], e


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_porosity_field(prec):
    case = workloads.grf_cavity(seed=1, n=128)
    _, _, e = run_pair(case["params"], 500, prec, phi=case["phi"], T=case["T"], C=case["C"])
    assert max(e.values()) <= TOL[prec], e


def test_full_size_grf_cavity_fp32():
    """512 x 512 Gaussian-random-field cavity in the benchmark launch shape, 200 steps."""
    case = workloads.grf_cavity(seed=1, n=512)
    _, _, e = run_pair(case["params"], 200, "fp32", phi=case["phi"], T=case["T"], C=case["C"])
    assert max(e.values()) <= TOL["fp32"], e


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_full_size_band_cavity(prec):
    """2048 x 2048 layered cavity (the benchmark workload), 20 steps, every node compared."""
    case = workloads.band_cavity(seed=2, n=2048)
    _, _, e = run_pair(case["params"], 20, prec, phi=case["phi"], T=case["T"], C=case["C"])
    print(prec, e, flush=True)
    assert max(e.values()) <= TOL[prec], e


@pytest.mark.parametrize("prec,nx,ny", [("fp32", 7500, 7482), ("fp64", 5300, 5319), ("fp16s", 10600, 10638)])
def test_largest_lattice(prec, nx, ny):
    """The largest lattice each storage type accepts: its 19 population planes just under the
    4 GiB range of one buffer resource, so the largest plane and lane offsets of the kernels
    are used.  Ragged tiles, a banded porosity field, 3 steps (a two-step launch, then a
    one-step launch), every node against the oracle.  FP16 storage: T, C and rho against the
    oracle within 1e-3 (a few stochastic roundings of deviations; the velocity after 3 steps
    from rest is too small for a relative bound), and bit for bit against one step per
    launch.  FP64: the largest speed after 3 steps is 3.3e-7, so the velocity is held to an
    absolute 1e-13 (the oracle sums O(1) populations, 9 per component, each rounded to
    1.1e-16, over 3 steps: a few 1e-15; measured 2e-16) instead of 1e-10 of the largest
    speed."""
    phi = np.repeat(0.35 + 0.07 * (np.arange(ny) * 8 // ny), nx).reshape(ny, nx)
    T, C = workloads.noise_fields(nx, ny, 21)
    p = workloads.cavity_params(nx=nx, ny=ny, Ra=1e6, Da=1e-3)
    gpu, ref, e = run_pair(p, 3, prec, phi=phi, T=T, C=C)
    if prec == "fp64":
        F, R = gpu.fields(), ref.fields()
        e["ux_abs"] = float(np.abs(F["ux"] - R["ux"]).max())
        e["uy_abs"] = float(np.abs(F["uy"] - R["uy"]).max())
        e["speed"] = float(np.hypot(R["ux"], R["uy"]).max())
        del F, R
    ref.close()
    print(prec, nx, ny, e, flush=True)
    if prec == "fp64":
        assert max(e["T"], e["C"], e["rho"]) <= TOL[prec] and max(e["ux_abs"], e["uy_abs"]) <= 1e-13, e
    elif prec == "fp16s":
        assert e["T"] < 1e-3 and e["C"] < 1e-3 and e["rho"] < 1e-3, e
        one = _solver()(p, phi=phi, T=T, C=C, precision=prec)
        one.set_steps_per_launch(1)
        one.step(3)
        d = _state_diff(one.get_state(), gpu.get_state())
        assert d is None, d
        one.close()
    else:
        assert max(e.values()) <= TOL[prec], e
    gpu.close()


def test_observables_parity():
    case = workloads.small_cavity(seed=0)
    p = case["params"]
    ref = Oracle(p, T=case["T"], C=case["C"])
    gpu = _solver()(p, T=case["T"], C=case["C"], precision="fp64")
    for steps in (300, 700):
        ref.step(steps)
        gpu.step(steps)
        a, b = gpu.observables(), ref.observables()
        for k in ("mass", "heat", "solute", "max_ux", "max_uy", "r_u", "r_T", "r_C"):
            assert a[k] == pytest.approx(b[k], rel=1e-10, abs=1e-14), k
        np.testing.assert_allclose(a["Nu"], b["Nu"], rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(a["Sh"], b["Sh"], rtol=1e-10, atol=1e-12)
        assert a["step"] == b["step"] and not a["nonfinite"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_moving_lid_and_horizontal_walls(prec):
    """Lid-driven cavity walls: moving top held hot, bottom cold, adiabatic sides."""
    p = workloads.cavity_params(nx=64, ny=48, sides=("adiabatic", "adiabatic", "cold", "hot"), Ra=1e4,
                                Le=1.0, N=2.0, phi=0.9, Da=1e-1, wall_u=(0.0, 0.0, 0.0, 0.05))
    _, _, e = run_pair(p, 600, prec, T=0.5, C=0.5)
    assert max(e.values()) <= TOL[prec], e


def test_periodic_channel_with_forcing():
    p = dict(nx=40, ny=24, sides=("adiabatic", "adiabatic", "periodic", "periodic"), direct=1, nu=0.05,
             alpha_e=0.04, D_e=0.02, K=30.0, gbT=1e-4, gbC=-5e-5, Fphi=0.5, phi=0.6, g_ext=(2e-5, 1e-4),
             Th=1.0, Tl=0.0)
    rng = np.random.default_rng(3)
    T = rng.uniform(0, 1, (24, 40))
    _, _, e = run_pair(p, 500, "fp64", T=T, C=1 - T)
    assert max(e.values()) <= 1e-10, e


def test_model_a():
    p = workloads.cavity_params(nx=48, ny=48, model=1, sigma=1.7, phi=0.6, Le=1.0)
    T, C = workloads.noise_fields(48, 48, 5)
    _, _, e = run_pair(p, 500, "fp64", T=T, C=C)
    assert max(e.values()) <= 1e-10, e


def test_nonzero_initial_velocity():
    p = workloads.cavity_params(nx=32, ny=32)
    rng = np.random.default_rng(8)
    ux = rng.uniform(-0.01, 0.01, (32, 32))
    uy = rng.uniform(-0.01, 0.01, (32, 32))
    _, _, e = run_pair(p, 200, "fp64", T=0.5, C=0.5, ux=ux, uy=uy)
    assert max(e.values()) <= 1e-10, e


def test_minimum_lattice():
    p = workloads.cavity_params(nx=3, ny=3)
    _, _, e = run_pair(p, 100, "fp64", T=0.5, C=0.5)
    assert max(e.values()) <= 1e-10, e


def test_degenerate_calls_and_smallest_lattices():
    """Zero steps change nothing; a negative count is refused; an empty batch steps as a no-op;
    the 3x3 lattice, with walls and periodic in one or both directions, gives the same state
    bit for bit with one, two and three steps per launch (three on FP32's 64 x 8 and 64 x 12
    tiles; tiles far wider than the lattice, halo nodes wrapped more than once across a periodic
    side)."""
    from paper_1708_07525_amd import Batch
    from paper_1708_07525_amd.lbm import LbmError
    Solver = _solver()
    p = workloads.cavity_params(nx=3, ny=3)
    s = Solver(p, T=0.5, C=0.5, precision="fp32")
    s.step(7)
    before = s.get_state()
    s.step(0)
    d = _state_diff(s.get_state(), before)
    assert d is None, d
    with pytest.raises(LbmError):
        s.step(-1)
    s.close()
    b = Batch(4, chunk=8)
    b.step(0)
    b.step(20)
    assert len(b) == 0
    b.close()
    for sides, g_ext in ((("cold", "hot", "adiabatic", "adiabatic"), (0.0, 0.0)),
                         (("periodic", "periodic", "cold", "hot"), (0.0, 0.0)),
                         (("periodic", "periodic", "periodic", "periodic"), (1e-5, 0.0))):
        for prec in ("fp32", "fp64"):
            pp = workloads.cavity_params(nx=3, ny=3, sides=sides, g_ext=g_ext)
            T, C = workloads.noise_fields(3, 3, 9)
            states = []
            for spl, rows in ((1, 0), (2, 0), (3, 8), (3, 12)):
                if rows == 12 and prec != "fp32":
                    continue
                sv = Solver(pp, T=T, C=C, precision=prec)
                sv.set_steps_per_launch(spl)
                sv.set_tile_rows(rows)
                sv.step(61)
                states.append(sv.get_state())
                sv.close()
            for st in states[1:]:
                d = _state_diff(st, states[0])
                assert d is None, (sides, prec, d)


# ------------------------------------------------------------ pins re-run on the GPU path

def test_gpu_linear_conduction_exact():
    eT, eC, Nu, Sh = pins.conduction_profile(make_gpu("fp64"))
    assert eT < 1e-12 and eC < 1e-12
    np.testing.assert_allclose(Nu + Sh, [1, 1, 1, 1], atol=1e-12)


def test_gpu_brinkman_poiseuille():
    assert pins.brinkman_poiseuille(make_gpu("fp64"), 32) < 1e-3
    # with the Forchheimer term of Eq. (5), against the finite-difference channel reference
    e16 = pins.brinkman_forchheimer_poiseuille(make_gpu("fp64"), 16)
    e32 = pins.brinkman_forchheimer_poiseuille(make_gpu("fp64"), 32)
    assert e32 < 1e-3 and 3.5 < e16 / e32 < 4.5, (e16, e32)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_gpu_d2q5_decay_equals_the_exact_step_operator(prec, tol):
    """The decay of a sine mode of T (sigma = 2) and of C (phi = 0.5) on the GPU path against the
    exact eigenvalue of the D2Q5 step operator, as in the oracle's pin."""
    assert abs(pins.sine_decay(make_gpu(prec), exact_operator=True, sigma=2.0)) < tol
    assert abs(pins.sine_decay(make_gpu(prec), exact_operator=True, phi=0.5, which="C")) < tol
    assert abs(pins.sine_decay(make_gpu(prec), exact_operator=True, sigma=2.0, u0=0.05)) < tol


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_gpu_d2q9_shear_wave_equals_the_exact_step_operator(prec, tol):
    assert abs(pins.shear_wave_decay(make_gpu(prec), A=1e-5 if prec == "fp64" else 1e-3)) < tol


def test_gpu_uniform_force_recurrence():
    err, got, closed = pins.uniform_force_history(make_gpu("fp64"), steps=50)
    assert err < 1e-14 and got == pytest.approx(closed, rel=1e-12)


def test_gpu_symmetry_and_conservation():
    assert pins.cavity_symmetry(make_gpu("fp64")) < 1e-12
    drifts, _ = pins.closed_box(make_gpu("fp64"), steps=1000)
    assert max(drifts) < 4 * np.finfo(float).eps * 1000


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s"])
def test_gpu_rest_state(prec):
    """In deviation form the rest state is all zeros and must stay exactly so."""
    worst, info = pins.rest_state(make_gpu(prec), detail=True)
    assert worst == 0.0, info


def test_gpu_buoyancy_cancellation():
    umax, dTC, Nu, Sh = pins.buoyancy_cancellation(make_gpu("fp32"))
    assert umax == 0.0 and dTC == 0.0 and Nu == Sh


# ------------------------------------------------------------ FP16 storage

def test_fp16s_error_bound():
    """Binary16 keeps 11 significant bits: each stored deviation is rounded (to nearest,
    unbiased) with relative error <= 2^-11, and the stored scalar deviations are at most
    |T - T0| <= 1/2.  A random walk of N such roundings bounds the scalar error by
    sqrt(N) 2^-11 / 2 = 7.7e-3 after N = 1000 steps.  The velocity, driven by the
    buoyancy of those scalars, is held to 2e-2 of the largest speed."""
    case = workloads.small_cavity(seed=0)
    _, _, e = run_pair(case["params"], 1000, "fp16s", T=case["T"], C=case["C"])
    print("fp16s", e, flush=True)
    bound = np.sqrt(1000) * 2.0 ** -11 / 2
    assert e["T"] < bound and e["C"] < bound and e["ux"] < 2e-2 and e["uy"] < 2e-2 and e["rho"] < 1e-3, e


def test_fp16s_error_bound_porosity_field():
    """FP16 storage on a Gaussian-random-field porosity cavity (96^2, 1000 steps): the bounds
    of test_fp16s_error_bound, with the concentration's divided by the smallest porosity
    (C = sum h / phi, so a rounding of h weighs 1/phi in C).  Measured: T, C 8e-4, u 1.4e-3."""
    case = workloads.grf_cavity(seed=1, n=96)
    _, _, e = run_pair(case["params"], 1000, "fp16s", phi=case["phi"], T=case["T"], C=case["C"])
    print("fp16s grf", e, flush=True)
    bound = np.sqrt(1000) * 2.0 ** -11 / 2
    assert e["T"] < bound and e["C"] < bound / float(case["phi"].min()), e
    assert e["ux"] < 2e-2 and e["uy"] < 2e-2 and e["rho"] < 1e-3, e


# ------------------------------------------------------------ launch-shape independence

def _state_after(steps, tile=None, prec="fp32", chunks=1):
    case = workloads.grf_cavity(seed=1, n=96)
    s = _solver()(case["params"], phi=case["phi"], T=case["T"], C=case["C"], precision=prec, tile=tile)
    for _ in range(chunks):
        s.step(steps // chunks)
    return s.get_state()


def test_results_do_not_depend_on_tile():
    ref = _state_after(50, (256, 1))
    for tile in ((64, 1), (128, 4), (64, 8), (256, 2)):
        d = _state_diff(_state_after(50, tile), ref)
        assert d is None, (tile, d)


@pytest.mark.parametrize("prec", ["fp32", "fp16s", "fp64"])
def test_results_do_not_depend_on_cache_policy(prec):
    Solver = _solver()
    case = workloads.grf_cavity(seed=1, n=96)
    states = []
    for policy in (-1, 0, 1, 2):
        s = Solver(case["params"], phi=case["phi"], T=case["T"], C=case["C"], precision=prec)
        s.set_cache_policy(policy)
        assert s.get_cache_policy() == (2 if policy == -1 else policy)   # 96^2 fits the cache: resident
        s.step(130)
        states.append(s.get_state())
        s.close()
    for st in states[1:]:
        d = _state_diff(st, states[0])
        assert d is None, d


@pytest.mark.parametrize("prec", ["fp32", "fp16s", "fp64"])
@pytest.mark.parametrize("case", ["grf_ragged", "lid_periodic", "nee_grf_ragged", "nee_lid_periodic"])
def test_two_step_kernel_matches_one_step(prec, case):
    """The LDS-staged two-step kernel against two launches of the one-step kernel, bitwise,
    on a ragged porosity-field cavity (tiles cut by every side) and on a channel periodic in
    x with a moving lid, each with half-way walls and with walls through the nodes (fixed,
    convective and zero-gradient sides; there the last tiles sit against the far walls and
    overlap their neighbours); the three-step kernel (FP32, FP64, half-way walls) too; step
    counts that are not multiples leave shorter launches; with and without graphs (a replay
    of 60 steps for three per launch).  FP16 storage with walls through the nodes always
    takes one step per launch."""
    Solver = _solver()
    if case.endswith("grf_ragged"):
        c = workloads.grf_cavity(seed=5, n=100)
        p, kw = dict(c["params"], ny=70), dict(phi=c["phi"][:70], T=c["T"][:70], C=c["C"][:70])
        if case.startswith("nee"):
            p.update(sides=("nee_hot", "nee_robin", "nee_adiabatic", "nee_cold"), Bi_T=2.0, Bi_C=0.5)
    else:
        sides = ("periodic", "periodic", "nee_cold", "nee_hot") if case.startswith("nee") else \
            ("periodic", "periodic", "cold", "hot")
        p = workloads.cavity_params(nx=70, ny=37, sides=sides, wall_u=(0.0, 0.0, 0.0, 0.05), Ra=5e4)
        T, C = workloads.noise_fields(70, 37, 8)
        kw = dict(T=T, C=C)
    states = {}
    for spl in (1, 2, 3):
        for chunk in (0, 64):
            s = Solver(p, precision=prec, **kw)
            s.set_steps_per_launch(spl)
            s.set_graph_chunk(chunk)
            expect = spl
            if spl == 3 and (prec == "fp16s" or case.startswith("nee")):
                expect = 2          # three steps per launch: FP32/FP64, half-way walls
            if prec == "fp16s" and case.startswith("nee"):
                expect = 1
            assert s.get_steps_per_launch() == expect
            s.step(131)
            s.step(70)
            states[(spl, chunk)] = s.get_state()
            s.close()
    ref = states[(1, 0)]
    for k, st in states.items():
        d = _state_diff(st, ref)
        assert d is None, (k, d)


@pytest.mark.parametrize("prec", ["fp32", "fp16s", "fp64"])
@pytest.mark.parametrize("walls", ["half_way", "nee", "periodic"])
def test_tile_order_changes_nothing(prec, walls):
    """The multi-step launches visit their tiles row by row or in vertical strips of k tiles
    (the last strip narrower), and FP32's three-step and FP16's two-step launches run on 64 x 8
    or 64 x 12 tiles:
    the state is the same bit for bit, on a wide ragged lattice
    (600 x 41: 10 tiles of 64 nodes across, 19 of 32 for FP64, a part-filled last row of
    tiles) with a porosity field, with half-way walls, walls through the nodes and periodic
    sides under a moving lid, with graph replays and plain launches."""
    Solver = _solver()
    nx, ny = 600, 41
    sides = {"half_way": ("hot", "cold", "adiabatic", "adiabatic"),
             "nee": ("nee_hot", "nee_cold", "nee_adiabatic", "nee_robin"),
             "periodic": ("periodic", "periodic", "cold", "hot")}[walls]
    lid = (0.0, 0.0, 0.0, 0.05 if walls == "periodic" else 0.0)       # a moving top wall
    p = workloads.cavity_params(nx=nx, ny=ny, sides=sides, Ra=5e4, Bi_T=2.0, Bi_C=0.5, wall_u=lid)
    phi = workloads.grf_porosity(nx, ny, 9, ell=8.0, lo=0.4, hi=0.9)
    T, C = workloads.noise_fields(nx, ny, 9)
    w = 32 if prec == "fp64" else 64
    ntx = (nx + w - 1) // w
    states = {}
    rows = (8, 12) if prec != "fp64" else (8,)
    for sw in (-1, 0, 1, 3, 4, 8, 64):
        for chunk in (0, 64):
            for r in rows:
                s = Solver(p, phi=phi, T=T, C=C, precision=prec)
                s.set_graph_chunk(chunk)
                s.set_strip_width(sw)
                s.set_tile_rows(r)
                assert s.get_tile_rows() == (8 if walls == "nee" else r)   # node walls: 8-row tiles
                if sw == -1:      # the default rule: row by row on a lattice that stays in the
                    assert s.get_strip_width() == 0              # Infinity Cache
                else:
                    assert s.get_strip_width() == sw
                s.step(131)
                states[(sw, chunk, r)] = s.get_state()
                s.close()
    ref = states[(0, 0, 8)]
    for k, st in states.items():
        d = _state_diff(st, ref)
        assert d is None, (k, d)


def test_launch_defaults_follow_the_lattice():
    """The default launch choices: FP32 three-step and FP16 two-step tiles of 12 rows where a
    step touches more than 400 MB (the lattice streams from HBM), 8 rows below and for FP64;
    there, one strip of tiles per XCD band when the tiles across are a multiple of 8, else
    strips of 8; row by row where the lattice stays in the Infinity Cache; invalid settings
    refused."""
    from paper_1708_07525_amd.lbm import LbmError
    Solver = _solver()
    for (nx, ny, prec), (rows, sw) in {(1460, 1460, "fp32"): (12, 8), (1456, 1460, "fp32"): (8, 0),
                                       (2100, 400, "fp32"): (8, 0), (500, 400, "fp32"): (8, 0),
                                       (1536, 1536, "fp32"): (12, 3), (3072, 800, "fp32"): (12, 6),
                                       (8192, 300, "fp32"): (12, 8), (2200, 1000, "fp32"): (12, 8),
                                       (1460, 1460, "fp64"): (8, 8), (1460, 1460, "fp16s"): (8, 0),
                                       (1900, 1900, "fp16s"): (12, 8), (2560, 1500, "fp16s"): (12, 5),
                                       (2048, 1200, "fp32"): (12, 4)}.items():
        s = Solver(workloads.cavity_params(nx=nx, ny=ny), T=0.5, C=0.5, precision=prec)
        assert (s.get_tile_rows(), s.get_strip_width()) == (rows, sw), (nx, ny, prec)
        with pytest.raises(LbmError):
            s.set_tile_rows(10)
        if prec == "fp64":
            with pytest.raises(LbmError):
                s.set_tile_rows(12)
        with pytest.raises(LbmError):
            s.set_strip_width(-2)
        s.close()


def test_graph_replays_match_plain_launches():
    """lbm_step uses a captured graph for chunks of 64 steps; replays interleaved with other
    work must give the same state as one launch per step."""
    ref = _state_after(192, chunks=192)          # steps of 1: plain launches only
    d = _state_diff(_state_after(192, chunks=1), ref)     # 3 graph replays
    assert d is None, d
    d = _state_diff(_state_after(192, chunks=3), ref)     # a replay per call
    assert d is None, d


def test_checkpoint_roundtrip():
    case = workloads.small_cavity(seed=0)
    p = case["params"]
    a = _solver()(p, T=case["T"], C=case["C"], precision="fp32")
    a.step(300)
    blob = a.get_state()
    a.step(300)
    b = _solver()(p, T=case["T"], C=case["C"], precision="fp32")
    b.set_state(blob)
    b.step(300)
    d = _state_diff(a.get_state(), b.get_state())
    assert d is None, d
    assert a.observables()["step"] == b.observables()["step"] == 600
    # a state whose header does not match the context (another lattice, or sizes altered) is
    # refused before anything is copied
    from paper_1708_07525_amd.lbm import LbmError
    import struct
    bad = bytearray(blob)
    hdr = 8 + 4 * 4 + 8 * 2               # magic, nx, ny, precision, counter, step, snap_step
    struct.pack_into("<Q", bad, hdr, struct.unpack_from("<Q", bad, hdr)[0] * 2)   # pop_bytes
    with pytest.raises(LbmError, match="does not match"):
        b.set_state(bytes(bad))
    d = _state_diff(a.get_state(), b.get_state())
    assert d is None, d


def test_unstable_is_reported():
    """A non-finite value is reported as LBM_EUNSTABLE; lbm_step then refuses with LBM_ESTATE
    until lbm_set_state gives the context a new state."""
    from paper_1708_07525_amd.lbm import ESTATE, EUNSTABLE, LbmError
    p = workloads.cavity_params(nx=16, ny=16)
    good = _solver()(p, T=0.5, C=0.5, precision="fp32")
    good.step(3)
    blob = good.get_state()
    T = np.full((16, 16), 0.5)
    T[3, 4] = np.nan
    s = _solver()(p, T=T, C=0.5, precision="fp32")
    s.step(3)
    ob = s.observables()
    assert ob["nonfinite"] and ob["status"] == EUNSTABLE
    with pytest.raises(LbmError) as ei:
        s.step(1)
    assert ei.value.status == ESTATE
    s.set_state(blob)
    s.step(2)
    good.step(2)
    d = _state_diff(s.get_state(), good.get_state())
    assert d is None, d


def test_lid_driven_mapping_on_the_device():
    """The section 4.3 mapping (Re, Gr, U0) of a context equals the host-only lbm_derive and
    the oracle's own mapping."""
    from paper_1708_07525_amd.lbm import derive
    p = workloads.cavity_params(nx=128, ny=128, sides=("adiabatic", "adiabatic", "cold", "hot"), direct=2,
                                Re=100.0, Gr=100.0, U0=0.1, Pr=1.0, Le=1.0, Da=0.1, N=-500.0, phi=0.95,
                                wall_u=(0.0, 0.0, 0.0, 0.1))
    s = _solver()(p, T=0.5, C=0.5, precision="fp64")
    d, h, o = s.derived(), derive(p, "fp64"), Oracle(p, T=0.5, C=0.5).derived()
    for k in ("nu", "s_v", "zeta_a", "eta_D", "gbT", "gbC", "K_mean", "U", "L"):
        assert d[k] == h[k], k
        assert d[k] == pytest.approx(o[k], rel=1e-14), k


# ------------------------------------------------------------ batching

def test_batch_alone_vs_mix_bitwise():
    from paper_1708_07525_amd import Batch
    Solver = _solver()
    specs = [
        (dict(workloads.cavity_params(nx=64, ny=64)), "fp32"),
        (dict(workloads.cavity_params(nx=96, ny=192, Ra=1e5, Le=4.0, N=-1.0, phi=0.5)), "fp32"),
        (dict(workloads.cavity_params(nx=70, ny=33, Ra=2e4, phi=0.8)), "fp16s"),
        (dict(workloads.cavity_params(nx=40, ny=40, Ra=5e3)), "fp64"),
        (dict(workloads.cavity_params(nx=128, ny=128, Ra=1e6, Da=1e-3, phi=0.4)), "fp32"),
    ]
    steps = 250    # two graph replays of 100 plus 50 single launches
    alone = []
    for i, (p, prec) in enumerate(specs):
        T, C = workloads.noise_fields(p["nx"], p["ny"], (7, i))
        s = Solver(p, T=T, C=C, precision=prec)
        s.step(steps)
        alone.append(s.get_state())
    mix = []
    b = Batch(len(specs), chunk=100)
    for i, (p, prec) in enumerate(specs):
        T, C = workloads.noise_fields(p["nx"], p["ny"], (7, i))
        s = Solver(p, T=T, C=C, precision=prec)
        b.attach(s)
        mix.append(s)
    b.step(steps)
    for s, ref in zip(mix, alone):
        d = _state_diff(s.get_state(), ref)
        assert d is None, d
    # detach one, keep going: the others are unaffected
    b.detach(mix[1])
    b.step(100)
    mix[1].step(100)
    assert len(b) == 4
    b.close()


def test_batch_member_closed_while_attached():
    """Destroying a context that is still attached detaches it first: the batch goes on with the
    others, which reach the states they reach alone, bit for bit."""
    from paper_1708_07525_amd import Batch
    Solver = _solver()
    specs = [workloads.cavity_params(nx=64, ny=48), workloads.cavity_params(nx=80, ny=80, Ra=1e5, phi=0.5)]
    fields = [workloads.noise_fields(p["nx"], p["ny"], (11, i)) for i, p in enumerate(specs)]
    alone = Solver(specs[1], T=fields[1][0], C=fields[1][1], precision="fp32")
    alone.step(350)
    ref = alone.get_state()
    alone.close()
    b = Batch(2, chunk=100)
    mix = [Solver(p, T=T, C=C, precision="fp32") for p, (T, C) in zip(specs, fields)]
    for s in mix:
        b.attach(s)
    b.step(250)
    mix[0].close()                       # not detached first
    assert len(b) == 1 and b.members == [mix[1]]
    b.step(100)
    d = _state_diff(mix[1].get_state(), ref)
    assert d is None, d
    b.close()
    mix[1].step(10)                      # back on its own stream
    mix[1].close()


@pytest.mark.parametrize("shape,chunk", [(0, 100), (1, 100), (2, 100), (3, 120), ("auto", 100), ("auto", 120)])
def test_batch_tile_shapes_change_nothing(shape, chunk):
    """Every tile shape of the batched two-step launch, three steps per launch (shape 3, FP32
    and FP64, with a chunk that is a multiple of 12), and the autotuner's choice give each
    cavity the state it reaches alone, bit for bit (cavities of all four size classes and the
    three storage types; widths that are not multiples of the tiles; two graph replays and a
    remainder of 8 steps: two three-step launches and two single steps)."""
    from paper_1708_07525_amd import Batch
    Solver = _solver()
    specs = [(workloads.cavity_params(nx=40, ny=52), "fp32"),
             (workloads.cavity_params(nx=96, ny=70, Ra=1e5, N=-1.0, phi=0.5), "fp32"),
             (workloads.cavity_params(nx=200, ny=100, Ra=3e4), "fp16s"),
             (workloads.cavity_params(nx=300, ny=45, Ra=2e4, Le=3.0), "fp64"),
             (workloads.cavity_params(nx=72, ny=72, Ra=5e3), "fp64"),
             # periodic in x with a moving lid: tiles wrapped across the periodic side
             (workloads.cavity_params(nx=70, ny=37, sides=("periodic", "periodic", "cold", "hot"),
                                      wall_u=(0.0, 0.0, 0.0, 0.05), Ra=5e4), "fp32"),
             (workloads.cavity_params(nx=70, ny=37, sides=("periodic", "periodic", "cold", "hot"),
                                      wall_u=(0.0, 0.0, 0.0, 0.05), Ra=5e4), "fp64"),
             # lattices smaller than one tile, walled and periodic
             (workloads.cavity_params(nx=5, ny=7, sides=("periodic", "periodic", "cold", "hot"), Ra=3e3), "fp32"),
             (workloads.cavity_params(nx=3, ny=3), "fp64"),
             (workloads.cavity_params(nx=6, ny=4), "fp16s")]
    steps = 2 * chunk + 8     # two replays and 8 more
    alone = []
    for i, (p, prec) in enumerate(specs):
        T, C = workloads.noise_fields(p["nx"], p["ny"], (11, i))
        s = Solver(p, T=T, C=C, precision=prec)
        s.step(steps)
        alone.append(s.get_state())
        s.close()
    b = Batch(len(specs), chunk=chunk)
    mix = []
    for i, (p, prec) in enumerate(specs):
        T, C = workloads.noise_fields(p["nx"], p["ny"], (11, i))
        s = Solver(p, T=T, C=C, precision=prec)
        b.attach(s)
        mix.append(s)
    if shape == "auto":
        chosen = b.autotune(8)
        print("batch autotune:", chosen, flush=True)
        assert set(chosen) == {("fp32", "<=64"), ("fp32", "<=128"), ("fp16s", "<=256"), ("fp64", ">256"),
                               ("fp64", "<=128"), ("fp64", "<=64"), ("fp16s", "<=64")}
    else:
        for prec in ("fp64", "fp32", "fp16s"):
            if shape == 3 and prec == "fp16s":
                with pytest.raises(RuntimeError):
                    b.set_tile(prec, 0, shape, -1)
                continue
            for cls in range(4):
                b.set_tile(prec, cls, shape, -1)
    b.step(steps)
    for s, ref in zip(mix, alone):
        d = _state_diff(s.get_state(), ref)
        assert d is None, (shape, s.nx, s.ny, s.precision, d)
    b.close()


def test_autotuned_tile_is_cached_and_changes_nothing(tmp_path, monkeypatch):
    from paper_1708_07525_amd import autotune
    monkeypatch.setenv("LBM_AUTOTUNE_CACHE", str(tmp_path / "tiles.json"))
    Solver = _solver()
    case = workloads.grf_cavity(seed=1, n=96)
    a = Solver(case["params"], phi=case["phi"], T=case["T"], C=case["C"], precision="fp32", tile="auto")
    assert len(autotune.load()) == 1
    b = Solver(case["params"], phi=case["phi"], T=case["T"], C=case["C"], precision="fp32", tile=(64, 8))
    a.step(50)
    b.step(50)
    d = _state_diff(a.get_state(), b.get_state())
    assert d is None, d


# ------------------------------------------------------------ walls through the nodes

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noisy_cavity_half_way_walls(prec):
    """The 40 x 36 cavity of the convective-wall test with half-way walls (hot, cold,
    adiabatic), Le = 1.5, N = 1, seed 21, 1000 steps, at the plain bars."""
    p = workloads.cavity_params(nx=40, ny=36, Ra=1e4, Da=1e-2, Le=1.5, N=1.0, phi=0.6)
    T, C = workloads.noise_fields(40, 36, 21)
    _, _, e = run_pair(p, 1000, prec, T=T, C=C)
    print(prec, e, flush=True)
    assert max(e.values()) <= TOL[prec], e


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("bi_c", [1.0, 200.0])
def test_convective_wall_cavity(prec, bi_c):
    p = workloads.cavity_params(nx=40, ny=36, sides=("nee_hot", "nee_robin", "nee_adiabatic", "nee_adiabatic"),
                                Ra=1e4, Da=1e-2, Le=1.5, N=1.0, phi=0.6, Bi_T=1.0, Bi_C=bi_c)
    T, C = workloads.noise_fields(40, 36, 21)
    gpu, ref, e = run_pair(p, 1000, prec, T=T, C=C)
    print(prec, e, flush=True)
    assert max(e.values()) <= TOL[prec], e
    a, b = gpu.observables(), ref.observables()
    np.testing.assert_allclose(a["Nu"], b["Nu"], rtol=10 * TOL[prec], atol=1e-12)
    np.testing.assert_allclose(a["Sh"], b["Sh"], rtol=10 * TOL[prec], atol=1e-12)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_extrapolation_walls_lid_and_porosity_field(prec):
    rng = np.random.default_rng(4)
    phi = rng.uniform(0.5, 0.9, size=(30, 34))
    p = workloads.cavity_params(nx=34, ny=30, sides=("nee_adiabatic", "nee_adiabatic", "nee_cold", "nee_hot"),
                                Ra=2e4, Da=5e-2, Le=2.0, N=-0.5, phi=0.7, wall_u=(0.0, 0.0, 0.0, 0.04))
    _, _, e = run_pair(p, 800, prec, phi=phi, T=0.5, C=0.5)
    assert max(e.values()) <= TOL[prec], e


def test_extrapolation_walls_periodic_channel():
    p = dict(nx=21, ny=8, sides=("nee_hot", "nee_cold", "periodic", "periodic"), direct=1, nu=0.05, alpha_e=0.04,
             D_e=0.02, K=30.0, gbT=1e-4, gbC=-5e-5, Fphi=0.5, phi=0.6, g_ext=(0.0, 1e-4))
    _, _, e = run_pair(p, 600, "fp64", T=0.5, C=0.5)
    assert max(e.values()) <= 1e-10, e


def test_fp16s_error_bound_node_walls():
    """The binary16 random-walk bound of test_fp16s_error_bound, on the convective-wall cavity
    with walls through the nodes (the boundary rebuild adds roundings of the same size)."""
    p = workloads.cavity_params(nx=40, ny=36, sides=("nee_hot", "nee_robin", "nee_adiabatic", "nee_adiabatic"),
                                Ra=1e4, Da=1e-2, Le=1.5, N=1.0, phi=0.6, Bi_T=1.0, Bi_C=2.0)
    T, C = workloads.noise_fields(40, 36, 21)
    _, _, e = run_pair(p, 1000, "fp16s", T=T, C=C)
    print("fp16s node walls", e, flush=True)
    bound = np.sqrt(1000) * 2.0 ** -11 / 2
    assert e["T"] < bound and e["C"] < bound and e["ux"] < 2e-2 and e["uy"] < 2e-2 and e["rho"] < 1e-3, e


def test_gpu_node_wall_pins():
    eT, eC, Nu, exact = pins.nee_conduction(make_gpu("fp64"))
    assert eT < 1e-12 and Nu == pytest.approx(exact, abs=1e-11)
    eT, eC, Nu, exact = pins.nee_conduction(make_gpu("fp64"), robin_bi=1.0)
    assert eT < 1e-11 and Nu == pytest.approx(exact, abs=1e-10)
    assert pins.nee_poiseuille(make_gpu("fp64"), 33) < 3e-3
    assert pins.cavity_symmetry(make_gpu("fp64"), sides=pins.NODE_CAVITY) < 1e-12
    e, uy = pins.couette_node_walls(make_gpu("fp64"))
    assert e < 1e-11 and uy < 1e-13


def test_gpu_couette_flow_is_exact():
    """The moving-wall term of the half-way bounce-back: the exact linear Couette profile on the
    GPU path (FP64), as in the oracle's pin."""
    e, uy = pins.couette(make_gpu("fp64"))
    assert e < 1e-11 and uy < 1e-13


@pytest.mark.parametrize("chunk,tune", [(100, False), (120, True)])
def test_batch_with_node_walls_alone_vs_mix(chunk, tune):
    """Cavities with walls through the boundary nodes (FP32 with a convective side, FP64) in a
    batch beside a plain cavity: each reaches the state it reaches alone, bit for bit.  The
    node-wall groups advance two steps per batched launch on tiles placed against the far
    walls; 2 replays and an odd remainder (the last single step is the cavity's own one-step
    launch).  With chunk 120 and the batch autotuner the plain cavity may take three steps per
    launch."""
    from paper_1708_07525_amd import Batch
    Solver = _solver()
    specs = [(workloads.cavity_params(nx=72, ny=40, sides=("nee_hot", "nee_robin", "nee_adiabatic", "nee_adiabatic"),
                                      Bi_T=1.0, Bi_C=5.0), "fp32"),
             (workloads.cavity_params(nx=64, ny=64), "fp32"),
             (workloads.cavity_params(nx=50, ny=50, sides=("nee_hot", "nee_cold", "nee_adiabatic", "nee_adiabatic")),
              "fp64"),
             (workloads.cavity_params(nx=130, ny=9, sides=("nee_hot", "nee_cold", "nee_adiabatic", "nee_adiabatic")),
              "fp32"),
             (workloads.cavity_params(nx=70, ny=37, sides=("periodic", "periodic", "nee_cold", "nee_hot"),
                                      wall_u=(0.0, 0.0, 0.0, 0.05), Ra=5e4), "fp32")]
    steps = 2 * chunk + 31
    alone = []
    for i, (p, prec) in enumerate(specs):
        T, C = workloads.noise_fields(p["nx"], p["ny"], (9, i))
        s = Solver(p, T=T, C=C, precision=prec)
        s.step(steps)
        alone.append(s.get_state())
        s.close()
    b = Batch(len(specs), chunk=chunk)
    mix = []
    for i, (p, prec) in enumerate(specs):
        T, C = workloads.noise_fields(p["nx"], p["ny"], (9, i))
        s = Solver(p, T=T, C=C, precision=prec)
        print(f"case nee-batch nx={s.nx} ny={s.ny} prec={prec} chunk={chunk}", flush=True)
        b.attach(s)
        mix.append(s)
    if tune:
        print("batch autotune:", b.autotune(12), flush=True)
    b.step(steps)
    for s, ref in zip(mix, alone):
        d = _state_diff(s.get_state(), ref)
        assert d is None, (s.nx, s.ny, s.precision, d)
    b.close()


def test_batch_refuses_node_walls():
    """Node-wall cavities the batch does not take: smaller than one two-step tile, FP16 storage,
    or a chunk that does not allow two steps per launch.  They still advance on their own."""
    from paper_1708_07525_amd import Batch
    from paper_1708_07525_amd.lbm import LbmError
    sides = ("nee_hot", "nee_cold", "nee_adiabatic", "nee_adiabatic")
    cases = [(workloads.cavity_params(nx=24, ny=24, sides=sides), "fp32", 12),
             (workloads.cavity_params(nx=80, ny=24, sides=sides), "fp16s", 12),
             (workloads.cavity_params(nx=80, ny=24, sides=sides), "fp32", 10)]
    for p, prec, chunk in cases:
        s = _solver()(p, T=0.5, C=0.5, precision=prec)
        b = Batch(2, chunk=chunk)
        with pytest.raises(LbmError, match="not batched"):
            b.attach(s)
        assert len(b) == 0
        s.step(10)                       # still advances on its own
        assert np.isfinite(s.fields()["T"]).all()
        b.close()
        s.close()
