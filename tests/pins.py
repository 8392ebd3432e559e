"""Measurements that pin a solver to what the paper and the mathematics fix.

Each function takes ``make(params, **fields)`` returning an object with ``step(n)``,
``fields()`` (dict of (ny, nx) arrays rho, ux, uy, T, C) and ``observables()``, so the
same pin runs on the FP64 oracle and on the GPU library.  Every reference value below
is computed from a closed form, a limit or an independent scalar recurrence, never by
re-running the solver's own formulas.
"""
import numpy as np

PERIODIC = ("periodic",) * 4
NO_FLOW = dict(direct=1, gbT=0.0, gbC=0.0, Fphi=0.0)


def conduction_profile(make, nx=16, ny=4, sigma=2.0, phi=0.7, steps=6000, **extra):
    """Pure conduction between a hot left and a cold right wall (no buoyancy): the
    steady profile is linear, T = Th + (Tl - Th)(x + 1/2)/nx with half-way walls, so the
    wall numbers are exactly 1.  Returns (max |T - exact|, max |C - exact|, Nu, Sh)."""
    p = dict(nx=nx, ny=ny, sides=("hot", "cold", "adiabatic", "adiabatic"), sigma=sigma, phi=phi,
             nu=0.1, alpha_e=0.2, D_e=0.1, K=1e30, **NO_FLOW)
    p.update(extra)
    s = make(p, T=0.5, C=0.5)
    s.step(steps)
    F = s.fields()
    x = np.arange(nx)
    exact = 1.0 - (x + 0.5) / nx
    ob = s.observables()
    return (np.abs(F["T"] - exact[None, :]).max(), np.abs(F["C"] - exact[None, :]).max(),
            ob["Nu"][:2], ob["Sh"][:2])


def brinkman_poiseuille(make, nx, J=2.0, nu=0.05, K16=50.0, phi=0.7, G=1e-5, steps=None, **extra):
    """Flow between no-slip walls at x = -1/2 and nx - 1/2, periodic in y, driven by a
    constant body acceleration G in y, without inertia (F_phi = 0).  Steady Brinkman
    equation nu_e u'' - (phi nu/K) u + phi G = 0 has the closed form
    u = (G K/nu) [1 - cosh(r (x - xc))/cosh(r nx/2)], r = sqrt(phi nu/(nu_e K)).
    K is scaled with nx^2 so that the profile shape is fixed.  Returns the relative L2
    error of u_y."""
    K = K16 * (nx / 16.0) ** 2
    p = dict(nx=nx, ny=3, sides=("adiabatic", "adiabatic", "periodic", "periodic"), J=J, phi=phi,
             nu=nu, alpha_e=0.1, D_e=0.1, K=K, g_ext=(0.0, G), **NO_FLOW)
    p.update(extra)
    s = make(p, T=0.5, C=0.5)
    s.step(steps or int(20 * nx * nx / (J * nu)))
    u = s.fields()["uy"][1]
    x = np.arange(nx)
    r = np.sqrt(phi * nu / (J * nu * K))
    ua = (G * K / nu) * (1.0 - np.cosh(r * (x - (nx - 1) / 2.0)) / np.cosh(r * nx / 2.0))
    return float(np.sqrt(((u - ua) ** 2).sum() / (ua ** 2).sum()))


def brinkman_forchheimer_reference(nx, nu_e, a, b, phiG, m=200):
    """Steady channel flow of Eq. (2) with the force of Eq. (5): nu_e u'' - a u - b |u| u + phi G
    = 0 between no-slip walls at x = -1/2 and nx - 1/2, by second-order finite differences on
    m points per lattice spacing, Newton's method, and one Richardson step between m and 2m;
    returns u at the nodes x = 0 .. nx - 1."""
    from scipy.linalg import solve_banded

    def solve(mm):
        n = nx * mm - 1                      # interior points; walls at both ends
        h = 1.0 / mm
        u = np.full(n, phiG / a)
        for _ in range(60):
            lap = np.empty(n)
            lap[1:-1] = u[:-2] - 2 * u[1:-1] + u[2:]
            lap[0] = -2 * u[0] + u[1]
            lap[-1] = u[-2] - 2 * u[-1]
            r = nu_e * lap / h ** 2 - a * u - b * np.abs(u) * u + phiG
            ab = np.zeros((3, n))
            ab[0, 1:] = nu_e / h ** 2
            ab[2, :-1] = nu_e / h ** 2
            ab[1, :] = -2 * nu_e / h ** 2 - a - 2 * b * np.abs(u)
            du = solve_banded((1, 1), ab, -r)
            u += du
            if np.abs(du).max() < 1e-15 * np.abs(u).max():
                break
        # node x_j = j sits at interior index (j + 1/2) mm - 1
        return u[[(j * mm + mm // 2) - 1 for j in range(nx)]]

    u1, u2 = solve(m), solve(2 * m)
    return u2 + (u2 - u1) / 3.0


def brinkman_forchheimer_poiseuille(make, nx, J=2.0, nu=0.05, K16=5.0, phi=0.7, G16=1e-4, F16=2.2,
                                    steps=None, **extra):
    """Channel flow as brinkman_poiseuille, with the Forchheimer term of Eq. (5): nu_e u'' -
    (phi nu/K) u - (phi F_phi/sqrt K) |u| u + phi G = 0.  K grows as nx^2, G as 1/nx^2 and F_phi as
    1/nx, so that the profile is the same at every nx: the channel is about four Brinkman
    lengths wide, and the Forchheimer drag lowers the core velocity from 0.0076 to 0.0056.
    Reference: brinkman_forchheimer_reference.  Returns the relative L2 error of u_y."""
    K = K16 * (nx / 16.0) ** 2
    G = G16 * (16.0 / nx) ** 2
    Fphi = F16 * 16.0 / nx
    p = dict(nx=nx, ny=3, sides=("adiabatic", "adiabatic", "periodic", "periodic"), J=J, phi=phi,
             nu=nu, alpha_e=0.1, D_e=0.1, K=K, g_ext=(0.0, G), direct=1, gbT=0.0, gbC=0.0, Fphi=Fphi)
    p.update(extra)
    s = make(p, T=0.5, C=0.5)
    s.step(steps or int(20 * nx * nx / (J * nu)))
    u = s.fields()["uy"][1]
    ua = brinkman_forchheimer_reference(nx, J * nu, phi * nu / K, phi * Fphi / np.sqrt(K), phi * G)
    return float(np.sqrt(((u - ua) ** 2).sum() / (ua ** 2).sum()))


def uniform_force_history(make, steps=200, phi=0.5, nu=0.05, K=20.0, Fphi=0.3, G=(6e-4, 2e-3), Fphi_ref=None,
                          **extra):
    """A fully periodic, spatially uniform state under a constant acceleration G.  Then
    streaming is the identity and the momentum obeys the trapezoidal recurrence
    u^{n+1} - F(u^{n+1})/2 = u^n + F(u^n)/2 with F(u) = -a u - b|u|u + phi G, a = phi nu/K,
    b = phi F_phi/sqrt(K) (Eq. 5); u^0 solves u - F(u)/2 = 0.  The recurrence is solved here
    by Newton's method.  Its fixed point F = 0 is the Darcy-Forchheimer velocity
    |u| = (-a + sqrt(a^2 + 4 b phi|G|))/(2b).
    Returns (max recurrence error over ``steps`` steps, |u| after 20000 more steps, the
    closed-form |u|).  ``Fphi_ref`` is the Forchheimer coefficient of the reference when the
    solver is given Fphi < 0 (the Ergun form of Eq. 7)."""
    p = dict(nx=3, ny=3, sides=PERIODIC, direct=1, nu=nu, alpha_e=0.1, D_e=0.1, K=K, gbT=0.0,
             gbC=0.0, Fphi=Fphi, phi=phi, g_ext=tuple(G))
    p.update(extra)
    s = make(p, T=0.5, C=0.5)
    a = phi * nu / K
    b = phi * (Fphi if Fphi_ref is None else Fphi_ref) / np.sqrt(K)
    Gv = np.array(G, dtype=float)

    def force(u):
        return -a * u - b * np.hypot(*u) * u + phi * Gv

    def solve(rhs):
        x = rhs.copy()
        for _ in range(60):
            r = x - force(x) / 2 - rhs
            n = np.hypot(*x)
            # Jacobian of x - F(x)/2
            Jm = np.eye(2) * (1 + a / 2 + b * n / 2)
            if n > 0:
                Jm += (b / 2) * np.outer(x, x) / n
            dx = np.linalg.solve(Jm, -r)
            x = x + dx
            if np.abs(dx).max() < 1e-19:
                break
        return x

    u = solve(np.zeros(2))
    err = 0.0
    for _ in range(steps):
        F = s.fields()
        got = np.array([F["ux"][1, 1], F["uy"][1, 1]])
        err = max(err, float(np.abs(got - u).max()))
        s.step(1)
        u = solve(u + force(u) / 2)
    s.step(20000)
    F = s.fields()
    got = float(np.hypot(F["ux"][1, 1], F["uy"][1, 1]))
    g = phi * np.hypot(*Gv)
    closed = (-a + np.sqrt(a * a + 4 * b * g)) / (2 * b) if b > 0 else g / a
    return err, got, float(closed)


def sine_decay(make, nx=64, sigma=1.0, phi=1.0, alpha=0.05, u0=0.0, which="T", t1=300, steps=2000,
               exact_operator=False, **extra):
    """A sine mode of T (or C) in a fully periodic domain, at rest or carried by a uniform
    flow u0 (no porous drag, no buoyancy).  Eqs. (3)-(4) give the amplitude decay rate
    alpha_e k^2/sigma (D_e k^2/phi) per step and the phase speed u0/sigma (u0/phi).
    Returns the relative error of the measured rate between steps t1 and t1 + steps, against
    that rate or, with exact_operator (at rest), against the exact rate of the discrete step
    (d2q5_mode_rate)."""
    p = dict(nx=nx, ny=3, sides=PERIODIC, nu=0.05, alpha_e=alpha, D_e=alpha, K=1e30, sigma=sigma,
             phi=phi, varpi=0.4, **NO_FLOW)
    p.update(extra)
    k = 2 * np.pi / nx
    x = np.arange(nx)
    prof = 0.5 + 0.1 * np.sin(k * x)[None, :].repeat(3, 0)
    s = make(p, T=prof, C=prof, ux=u0)
    key = "T" if which == "T" else "C"
    cap = sigma if which == "T" else phi

    def amp():
        return np.abs(np.fft.fft(s.fields()[key][1] - 0.5)[1])

    s.step(t1)
    a0 = amp()
    s.step(steps)
    a1 = amp()
    rate = -np.log(a1 / a0) / steps
    if exact_operator:
        return float(rate / d2q5_mode_rate(nx, cap, p["varpi"], alpha, u0) - 1.0)
    return float(rate / (alpha * k * k / cap) - 1.0)


def d2q5_mode_rate(nx, cap, varpi, diff, u0=0.0, rate_e=1.5, rate_eps=1.5):
    """Exact per-step decay rate of the slowest sine mode (wavenumber 2 pi/nx along x) of the
    D2Q5 scheme, present model, in a uniform flow u0 along x (0: at rest).  The state of the
    mode is its 5 population amplitudes and the previous step's T (kept for Eq. 27); one step is
    the moment-space collision of Eqs. (21)-(22) with the source term,
    n* = n - Theta (n - n^eq) + (I - Theta/2) (0, u0 (T - T_prev), 0, 0, 0),
    n^eq = (cap T, u0 T, 0, (5 varpi - 4 cap) T, 0) (Eq. 24), T = sum g/cap (cap = sigma for g,
    phi for h), N of Eq. (23), Theta = diag(1, z, z, rate_e, rate_eps) with z = 1/(1/2 +
    diff/(varpi/2)) (Eq. 29), followed by pull streaming (phase exp(-i k e_x) per direction).
    Returns -ln of the modulus of the step operator's eigenvalue of largest modulus."""
    N = np.array([[1, 1, 1, 1, 1], [0, 1, 0, -1, 0], [0, 0, 1, 0, -1], [-4, 1, 1, 1, 1], [0, 1, -1, 1, -1]],
                 dtype=float)
    Ni = np.linalg.inv(N)
    z = 1.0 / (0.5 + diff / (varpi / 2.0))
    th = np.diag([1.0, z, z, rate_e, rate_eps])
    t = np.ones((1, 5)) / cap                                  # T = t g
    q = np.array([[cap], [u0], [0.0], [5 * varpi - 4 * cap], [0.0]])
    src = (np.eye(5) - th / 2) @ np.array([[0.0], [u0], [0.0], [0.0], [0.0]])
    k = 2 * np.pi / nx
    P = np.diag(np.exp(-1j * k * np.array([0, 1, 0, -1, 0])))
    A = np.zeros((6, 6), dtype=complex)
    A[:5, :5] = P @ Ni @ ((np.eye(5) - th) @ N + th @ q @ t + src @ t)
    A[:5, 5:] = P @ Ni @ (-src)
    A[5:, :5] = t
    lam = np.linalg.eigvals(A)
    return float(-np.log(np.abs(lam).max()))


def d2q9_shear_rate(nx, nu_e, rates=(1.0, 1.1, 1.1, 1.0, 1.2, 1.0, 1.2), rho0=1.0):
    """Exact per-step decay rate of a shear wave u_y = A sin(2 pi x/nx) of the D2Q9 scheme at
    small amplitude, without drag or force: the linear step operator on the mode's 9 population
    amplitudes is pull streaming after the moment-space collision of Eq. (10),
    f* = f - M^-1 S M (f - f^eq), with M built from the Lallemand-Luo polynomials (Eq. 13), the
    equilibrium of Eq. (20) to first order in u, w_i (rho + rho0 3 e_i.u) with u = j/rho0 (Eqs.
    17-19 with no drag), and S = diag(s_rho, s_e, s_eps, s_j, s_q, s_j, s_q, s_v, s_v), s_v =
    1/(1/2 + 3 nu_e) (section 2.2).  `rates` are (s_rho, s_e, s_eps, s_j, s_q, s_j, s_q).
    Returns -ln of the modulus of the eigenvalue of the shear mode (the eigenvector that carries
    j_y)."""
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
    ey = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    e2 = ex ** 2 + ey ** 2
    M = np.array([np.ones(9), -4 + 3 * e2, 4 - 10.5 * e2 + 4.5 * e2 ** 2, ex, (-5 + 3 * e2) * ex, ey,
                  (-5 + 3 * e2) * ey, ex ** 2 - ey ** 2, ex * ey])
    sv = 1.0 / (0.5 + 3.0 * nu_e)
    S = np.diag(list(rates) + [sv, sv])
    E = np.outer(w, np.ones(9)) + 3 * np.outer(w * ex, ex) + 3 * np.outer(w * ey, ey)
    k = 2 * np.pi / nx
    P = np.diag(np.exp(-1j * k * ex))
    A = P @ (np.eye(9) - np.linalg.solve(M, S @ M) @ (np.eye(9) - E))
    lam, vec = np.linalg.eig(A)
    jy = np.abs(ey @ vec) / np.linalg.norm(vec, axis=0)
    return float(-np.log(np.abs(lam[np.argmax(jy)])))


def shear_wave_decay(make, nx=64, nu=0.05, J=1.0, A=1e-5, t1=400, steps=2000, **extra):
    """A shear wave u_y = A sin(2 pi x/nx) in a fully periodic domain without drag, force or
    buoyancy: the measured per-step decay rate of its amplitude between steps t1 and
    t1 + steps, relative to the exact rate of the linear step operator (d2q9_shear_rate), minus
    one."""
    p = dict(nx=nx, ny=3, sides=PERIODIC, nu=nu, J=J, alpha_e=0.05, D_e=0.05, K=1e30, phi=0.8, **NO_FLOW)
    p.update(extra)
    k = 2 * np.pi / nx
    uy = A * np.sin(k * np.arange(nx))[None, :].repeat(3, 0)
    s = make(p, T=0.5, C=0.5, uy=uy)

    def amp():
        return np.abs(np.fft.fft(s.fields()["uy"][1])[1])

    s.step(t1)
    a0 = amp()
    s.step(steps)
    a1 = amp()
    rate = -np.log(a1 / a0) / steps
    return float(rate / d2q9_shear_rate(nx, J * nu) - 1.0)


def sine_phase_speed(make, nx=128, sigma=2.0, u0=0.05, steps=400, **extra):
    """Phase speed of an advected sine mode of T relative to u0/sigma (Eq. 3)."""
    p = dict(nx=nx, ny=3, sides=PERIODIC, nu=0.05, alpha_e=0.05, D_e=0.05, K=1e30, sigma=sigma,
             phi=1.0, varpi=0.4, **NO_FLOW)
    p.update(extra)
    k = 2 * np.pi / nx
    x = np.arange(nx)
    prof = 0.5 + 0.1 * np.sin(k * x)[None, :].repeat(3, 0)
    s = make(p, T=prof, C=prof, ux=u0)
    s.step(100)
    ph0 = np.angle(np.fft.fft(s.fields()["T"][1] - 0.5)[1])
    s.step(steps)
    ph1 = np.angle(np.fft.fft(s.fields()["T"][1] - 0.5)[1])
    dph = (ph0 - ph1) % (2 * np.pi)
    return float((dph / k / steps) / (u0 / sigma) - 1.0)


def closed_box(make, nx=24, ny=20, steps=2000, seed=5, **extra):
    """All four sides adiabatic and no-slip, random porosity and initial T, C, buoyancy
    on.  Mass, heat and solute (sum rho, sum sigma T, sum phi C) are invariant.
    Returns the relative drifts."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.45, 0.9, size=(ny, nx))
    T = rng.uniform(0.0, 1.0, size=(ny, nx))
    C = rng.uniform(0.0, 1.0, size=(ny, nx))
    p = dict(nx=nx, ny=ny, sides=("adiabatic",) * 4, Ra=1e5, Da=1e-2, Le=3.0, N=0.7, sigma=1.3,
             phi=0.6)
    p.update(extra)
    s = make(p, phi=phi, T=T, C=C)
    o0 = s.observables()
    s.step(steps)
    o1 = s.observables()
    return tuple(abs(o1[k] - o0[k]) / abs(o0[k]) for k in ("mass", "heat", "solute")), o1


def rest_state(make, nx=12, ny=10, steps=300, detail=False, **extra):
    """u = 0 and T = C = 0.5 everywhere, walls held at the same values: the state must not
    move.  Returns max |field - initial| over (rho - rho0, u, T, C) (with ``detail``, also
    the per-field maxima and the first offending nodes)."""
    p = dict(nx=nx, ny=ny, sides=("hot", "cold", "adiabatic", "adiabatic"), Th=0.5, Tl=0.5,
             Ch=0.5, Cl=0.5, direct=1, nu=0.05, alpha_e=0.05, D_e=0.03, K=30.0, gbT=1e-3,
             gbC=-2e-4, Fphi=-1.0, phi=0.55)
    p.update(extra)
    s = make(p, T=0.5, C=0.5)
    s.step(steps)
    F = s.fields()
    ref = dict(rho=1.0, ux=0.0, uy=0.0, T=0.5, C=0.5)
    errs = {k: np.abs(F[k] - ref[k]) for k in ref}
    worst = max(float(e.max()) for e in errs.values())
    if detail:
        info = {k: (float(e.max()), np.argwhere(e > 0)[:4].tolist()) for k, e in errs.items()}
        return worst, info
    return worst


def cavity_symmetry(make, nx=32, ny=24, steps=2000, **extra):
    """A noise-free cavity with uniform porosity, hot left and cold right walls and
    scalars centred on zero (walls at +-1/2, initial T = C = 0): rotating the domain by
    pi maps the discrete problem onto itself with T -> -T, C -> -C, u -> -u, because the
    D2Q5 equilibria, the source term and the buoyancy are all linear in the scalars.
    (A shifted scalar, T -> 1 - T, is not an exact symmetry of the lattice scheme: the
    equilibrium flux u T transports a constant only where the lattice divergence of u
    vanishes.)  Returns the largest violation."""
    p = dict(nx=nx, ny=ny, Ra=5e4, Da=1e-2, Le=2.0, N=0.5, phi=0.6, Th=0.5, Tl=-0.5, Ch=0.5, Cl=-0.5)
    p.update(extra)
    s = make(p, T=0.0, C=0.0)
    s.step(steps)
    F = s.fields()
    rot = lambda a: a[::-1, ::-1]
    scale = max(np.abs(F["ux"]).max(), np.abs(F["uy"]).max())
    return max(float(np.abs(F["T"] + rot(F["T"])).max()), float(np.abs(F["C"] + rot(F["C"])).max()),
               float(np.abs(F["ux"] + rot(F["ux"])).max() / scale),
               float(np.abs(F["uy"] + rot(F["uy"])).max() / scale),
               float(np.abs(F["rho"] - rot(F["rho"])).max()))


def hot_fluid_rises(make, nx=32, ny=32, steps=1500, **extra):
    """Eq. (6) with j pointing up: next to the hot left wall the fluid rises (u_y > 0)
    and next to the cold right wall it sinks.  Returns (mean u_y of the first column,
    mean u_y of the last column)."""
    p = dict(nx=nx, ny=ny, Ra=1e5, Da=1e-1, Le=1.0, N=0.0, phi=0.8)
    p.update(extra)
    s = make(p, T=0.5, C=0.5)
    s.step(steps)
    F = s.fields()
    return float(F["uy"][:, 0].mean()), float(F["uy"][:, -1].mean())


def le1_decoupling(make, n=24, steps=40000, sigma=2.0, phi=0.6, model=0, **extra):
    """Le = 1 with identical walls and initial fields for T and C and sigma != phi: the
    present model's steady state has T = C, hence Nu = Sh (section 3.2 and Tables 3 and
    5); Model-A's does not.  Returns (max |T - C|, Nu - Sh, r_u)."""
    p = dict(nx=n, ny=n, Ra=1e3, Pr=1.0, Le=1.0, Da=1e-2, N=1.0, sigma=sigma, phi=phi, model=model)
    p.update(extra)
    s = make(p, T=0.5, C=0.5)
    s.step(steps - 1000)
    s.observables()
    s.step(1000)
    ob = s.observables()
    F = s.fields()
    return float(np.abs(F["T"] - F["C"]).max()), ob["Nu"][0] - ob["Sh"][0], ob["r_u"]


def buoyancy_cancellation(make, n=20, steps=1500, seed=9, **extra):
    """Le = 1, N = -1, sigma = phi and T, C started from the same noisy field: T and C
    evolve identically, so the buoyancy of Eq. (6) vanishes and the fluid never moves.
    Returns (max |u|, max |T - C|, Nu, Sh at the hot wall)."""
    rng = np.random.default_rng(seed)
    T = 0.5 + rng.uniform(-1e-2, 1e-2, size=(n, n))
    p = dict(nx=n, ny=n, Ra=1e5, Pr=1.0, Le=1.0, Da=1e-1, N=-1.0, sigma=0.7, phi=0.7)
    p.update(extra)
    s = make(p, T=T, C=T.copy())
    s.step(steps)
    F = s.fields()
    ob = s.observables()
    return (float(max(np.abs(F["ux"]).max(), np.abs(F["uy"]).max())), float(np.abs(F["T"] - F["C"]).max()),
            ob["Nu"][0], ob["Sh"][0])


# ------------------------------------------------------------------ walls through the nodes

NODE_CAVITY = ("nee_hot", "nee_cold", "nee_adiabatic", "nee_adiabatic")


def nee_conduction(make, nx=12, ny=6, sigma=1.5, phi=0.7, steps=8000, robin_bi=None, **extra):
    """Conduction with walls through the boundary nodes (Eqs. 33-37): hot left wall; right
    wall cold, or convective with Biot number Bi (Eq. 39, flux out = Bi/L (T_b - T_inf), with
    L = nx - 1 the wall-to-wall width and T_inf = Tl); zero-flux top and bottom.  The steady
    profile is linear and the schemes are exact for it: T = Th - (Th - T_R) x/(nx - 1) with
    T_R = Tl, or T_R = (Th + Bi T_inf)/(1 + Bi).  Returns (max |T - exact|, max |C - exact|,
    Nu at the left, the exact Nu)."""
    sides = ("nee_hot", "nee_robin" if robin_bi is not None else "nee_cold", "nee_adiabatic", "nee_adiabatic")
    p = dict(nx=nx, ny=ny, sides=sides, sigma=sigma, phi=phi, nu=0.1, alpha_e=0.15, D_e=0.1, K=1e30,
             Bi_T=robin_bi or 0.0, Bi_C=robin_bi or 0.0, **NO_FLOW)
    p.update(extra)
    s = make(p, T=0.5, C=0.5)
    s.step(steps)
    F = s.fields()
    TR = 0.0 if robin_bi is None else 1.0 / (1.0 + robin_bi)
    exact = 1.0 - (1.0 - TR) * np.arange(nx) / (nx - 1)
    ob = s.observables()
    return (float(np.abs(F["T"] - exact[None, :]).max()), float(np.abs(F["C"] - exact[None, :]).max()),
            ob["Nu"][0], 1.0 - TR)


def nee_poiseuille(make, nx, J=2.0, nu=0.05, K16=50.0, phi=0.7, G=1e-5, steps=None, **extra):
    """Brinkman channel flow with no-slip walls through the nodes x = 0 and x = nx - 1
    (u_b = 0 imposed by Eq. 33), periodic in y; closed form with width W = nx - 1:
    u = (G K/nu) [1 - cosh(r (x - W/2))/cosh(r W/2)].  Returns the relative L2 error."""
    K = K16 * (nx / 16.0) ** 2
    p = dict(nx=nx, ny=3, sides=("nee_adiabatic", "nee_adiabatic", "periodic", "periodic"), J=J, phi=phi,
             nu=nu, alpha_e=0.1, D_e=0.1, K=K, g_ext=(0.0, G), **NO_FLOW)
    p.update(extra)
    s = make(p, T=0.5, C=0.5)
    s.step(steps or int(20 * nx * nx / (J * nu)))
    u = s.fields()["uy"][1]
    x = np.arange(nx)
    W = nx - 1
    r = np.sqrt(phi * nu / (J * nu * K))
    ua = (G * K / nu) * (1.0 - np.cosh(r * (x - W / 2.0)) / np.cosh(r * W / 2.0))
    return float(np.sqrt(((u - ua) ** 2).sum() / (ua ** 2).sum()))


def couette(make, ny=16, U=0.01, phi=0.7, nu=0.1, steps=20000, **extra):
    """Plane Couette flow: x periodic, a no-slip bottom wall at y = -1/2 and a top wall at
    y = ny - 1/2 moving with U (the moving-wall term of the half-way bounce-back), no force
    and no drag.  The steady profile is linear, u_x = U (y + 1/2)/ny, and the scheme is exact
    for it.  Returns max |u_x - exact| / U and max |u_y|."""
    p = dict(nx=3, ny=ny, sides=("periodic", "periodic", "adiabatic", "adiabatic"), wall_u=(0.0, 0.0, 0.0, U),
             phi=phi, nu=nu, alpha_e=0.1, D_e=0.1, K=1e30, **NO_FLOW)
    p.update(extra)
    s = make(p, T=0.5, C=0.5)
    s.step(steps)
    F = s.fields()
    exact = U * (np.arange(ny) + 0.5) / ny
    return float(np.abs(F["ux"] - exact[:, None]).max() / U), float(np.abs(F["uy"]).max())


def couette_node_walls(make, ny=17, U=0.01, phi=0.7, nu=0.1, steps=20000, **extra):
    """Plane Couette flow between walls through the first and last rows of nodes (Eqs. 33-35):
    x periodic, the bottom row at rest, the top row moving with U (the wall velocity in the
    equilibrium of Eq. 33), no force and no drag.  The steady profile is linear through the
    nodes, u_x = U y/(ny - 1), and the extrapolation is exact for it (the non-equilibrium part
    of a linear profile is the same at every node).  Returns max |u_x - exact| / U and
    max |u_y|."""
    p = dict(nx=3, ny=ny, sides=("periodic", "periodic", "nee_adiabatic", "nee_adiabatic"),
             wall_u=(0.0, 0.0, 0.0, U), phi=phi, nu=nu, alpha_e=0.1, D_e=0.1, K=1e30, **NO_FLOW)
    p.update(extra)
    s = make(p, T=0.5, C=0.5)
    s.step(steps)
    F = s.fields()
    exact = U * np.arange(ny) / (ny - 1)
    return float(np.abs(F["ux"] - exact[:, None]).max() / U), float(np.abs(F["uy"]).max())


def layered_darcy(make, nx=80, ny=3, phis=(0.4, 0.8), K_mean=1.0, nu=0.05, G=1e-5, steps=3000, **extra):
    """Flow along two porous layers (x < nx/2 and x >= nx/2, periodic in x and y), driven by a
    constant acceleration G along y, without Forchheimer term.  Far from the interface each
    layer carries the Darcy velocity u = G K/nu of its own permeability (Eq. 5 with the
    Brinkman term negligible: the layers are 20 Brinkman lengths wide or more).  Returns, per
    layer, the measured velocity at its centre over G K/nu - 1 with K(phi) from the
    Kozeny-Carman form of Eq. (7) scaled so that its mean over the lattice is K_mean."""
    phi = np.where(np.arange(nx) < nx // 2, phis[0], phis[1])[None, :].repeat(ny, 0)
    p = dict(nx=nx, ny=ny, sides=PERIODIC, direct=1, nu=nu, alpha_e=0.1, D_e=0.1, K=K_mean, gbT=0.0,
             gbC=0.0, Fphi=0.0, phi=0.6, g_ext=(0.0, G))
    p.update(extra)
    s = make(p, phi=phi, T=0.5, C=0.5)
    s.step(steps)
    u = s.fields()["uy"][ny // 2]
    kc = [q ** 3 / (1 - q) ** 2 for q in phis]
    mean = (kc[0] + kc[1]) / 2
    return [float(u[xc] / (G * K_mean * k / mean / nu) - 1.0) for xc, k in ((nx // 4, kc[0]), (3 * nx // 4, kc[1]))]
