"""The GPU path against the numbers the paper prints (section 4): Table 1 (pure-fluid
enclosure, the hot-path wall types) and Tables 4-5 (lid-driven porous cavity: moving-lid
bounce-back, horizontal hot/cold walls, Re-based viscosity).  The paper's walls are
non-equilibrium extrapolation; with half-way bounce-back the agreement is at the level of
the discretisation, and the bars below are stated per case."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def run_to_steady(s, chunk=5000, tol=1e-9, cap=400000, scalars=False):
    """Step until the velocity residual (and, with ``scalars``, the T and C residuals) per
    step falls below tol, or the cap."""
    s.observables()
    steps = 0
    while steps < cap:
        s.step(chunk)
        steps += chunk
        ob = s.observables()
        r = max(ob["r_u"], ob["r_T"], ob["r_C"]) if scalars else ob["r_u"]
        if r < tol:
            break
    return ob, steps


def lid_driven_params(N, phi=0.95, model=0, n=128, Gr=1e2, Re=100.0, Da=0.1, Pr=1.0, Le=1.0, U0=0.1):
    """Section 4.3: nu = U0 L/Re (1/s_v = 1/2 + J L U0/(c_s^2 Re)), alpha_e = nu/Pr,
    D_e = alpha_e/Le, K = Da L^2, g beta_T dT = Gr nu^2/L^3, beta_C dC = N beta_T dT."""
    nu = U0 * n / Re
    gbT = Gr * nu * nu / n ** 3
    return dict(nx=n, ny=n, sides=("adiabatic", "adiabatic", "cold", "hot"), direct=1, nu=nu, alpha_e=nu / Pr,
                D_e=nu / Pr / Le, K=Da * n * n, gbT=gbT, gbC=N * gbT, phi=phi, model=model,
                wall_u=(0.0, 0.0, 0.0, U0), Th=1.0, Tl=0.0, Ch=1.0, Cl=0.0)


def test_table1_pure_fluid_enclosure():
    from paper_1708_07525_amd import Solver
    ref = json.load(open(os.path.join(GOLDEN, "table1_pure_fluid_enclosure.json")))["quantities"]
    p = dict(nx=100, ny=200, Ra=1e5, Pr=1.0, Le=2.0, Da=1e8, N=-0.8, phi=1.0)
    s = Solver(p, T=0.5, C=0.5, precision="fp64")
    ob, steps = run_to_steady(s, chunk=10000, tol=1e-8, cap=400000)
    scale = 100 / s.derived()["alpha_e"]
    got = dict(Nu=ob["Nu"][0], Sh=ob["Sh"][0], ux=ob["max_ux"] * scale, uy=ob["max_uy"] * scale)
    print("table 1:", got, "steps", steps, "r_u", ob["r_u"], flush=True)
    assert got["Nu"] == pytest.approx(ref["Nu_left"], rel=0.02)
    assert got["Sh"] == pytest.approx(ref["Sh_left"], rel=0.02)
    assert got["ux"] == pytest.approx(ref["max_abs_ux_in_alpha_e_over_L"], rel=0.02)
    assert got["uy"] == pytest.approx(ref["max_abs_uy_in_alpha_e_over_L"], rel=0.02)


def test_table4_lid_driven_nu_sh():
    from paper_1708_07525_amd import Solver
    ref = json.load(open(os.path.join(GOLDEN, "table4_lid_driven.json")))
    rows = []
    for N, nu_ref in zip(ref["N"], ref["Nu_bottom"]):
        s = Solver(lid_driven_params(N), T=0.5, C=0.5, precision="fp64")
        ob, steps = run_to_steady(s, chunk=5000, tol=1e-10, cap=600000, scalars=True)
        rows.append((N, ob["Nu"][2], ob["Sh"][2], nu_ref, steps))
        print(f"table 4: N={N} Nu={ob['Nu'][2]:.4f} Sh={ob['Sh'][2]:.4f} paper={nu_ref} steps={steps}", flush=True)
        s.close()
    for N, Nu, Sh, nu_ref, _ in rows:
        assert Nu == pytest.approx(Sh, rel=1e-6), N           # Le = 1: identical steady fields
        assert Nu == pytest.approx(nu_ref, rel=0.03), N


def test_table5_present_vs_model_a():
    """phi = 0.6: the present model keeps Nu = Sh; Model-A (Eqs. 30-32) splits them."""
    from paper_1708_07525_amd import Solver
    ref = json.load(open(os.path.join(GOLDEN, "table4_lid_driven.json")))["table5_phi0.6"]
    for N in (-1500, -500):
        res = {}
        for model in (0, 1):
            s = Solver(lid_driven_params(N, phi=0.6, model=model), T=0.5, C=0.5, precision="fp64")
            ob, steps = run_to_steady(s, chunk=5000, tol=1e-10, cap=600000, scalars=True)
            res[model] = (ob["Nu"][2], ob["Sh"][2], steps)
            s.close()
        print(f"table 5: N={N} present={res[0]} model-A={res[1]} paper={ref[f'N={N}']}", flush=True)
        p_nu, p_sh = ref[f"N={N}"]["present"]
        assert res[0][0] == pytest.approx(res[0][1], rel=1e-6)
        assert res[0][0] == pytest.approx(p_nu, rel=0.03)
        # Model-A's artificial coupling leaves Nu != Sh, by 1e-4 or more as in Table 5
        assert abs(res[1][0] - res[1][1]) > 1e-4 * abs(res[1][0])
