"""Bookkeeping of the continuous-batching loop, on the CPU with a stand-in backend.

The stand-in cavity relaxes its 'velocity' geometrically with a rate set by its
parameters, so the residual check, the step cap, admission under the memory budget,
slot reuse and the alone-versus-mixed equality can be checked without a GPU.
"""
import numpy as np
import pytest

from paper_1708_07525_amd.serving import Request, Server, converged


class FakeSolver:
    live = 0

    def __init__(self, params, phi=None, T=None, C=None, precision="fp32"):
        self.nx, self.ny = params["nx"], params["ny"]
        self.rate = params["rate"]
        self.node_walls = any(str(k).startswith("nee_") for k in params.get("sides", ()))
        self.u = 1.0
        self.step_n = 0
        self.snap_u = self.u
        self.snap_step = 0
        self.closed = False
        FakeSolver.live += 1

    def advance(self, n):
        self.u *= (1 - self.rate) ** n
        self.step_n += n

    def step(self, n):          # a cavity stepped outside the batch
        self.advance(n)

    def observables(self):
        dn = self.step_n - self.snap_step
        r = abs(self.u - self.snap_u) / (max(dn, 1) * max(self.u, 1e-30))
        self.snap_u, self.snap_step = self.u, self.step_n
        return dict(max_ux=self.u, max_uy=0.0, r_u=r, r_T=0.0, r_C=0.0, nonfinite=False, step=self.step_n)

    def derived(self):
        return dict(U=1.0)

    def fields(self):
        return dict(u=self.u)

    def close(self):
        assert not self.closed
        self.closed = True
        FakeSolver.live -= 1


class FakeBatch:
    def __init__(self, cap, chunk):
        self.cap, self.chunk, self.members = cap, chunk, []

    def attach(self, s):
        assert len(self.members) < self.cap
        if s.node_walls and s.nx < 64:      # as the library: too small for a two-step tile
            from paper_1708_07525_amd.lbm import EINVAL, LbmError
            raise LbmError(EINVAL, "walls through the boundary nodes on a small lattice are not batched")
        self.members.append(s)

    def detach(self, s):
        self.members.remove(s)

    def step(self, n):
        for s in self.members:
            s.advance(n)

    def close(self):
        pass


class FakeBackend:
    Solver = FakeSolver
    Batch = FakeBatch

    @staticmethod
    def footprint_bytes(params, precision):
        return params["nx"] * params["ny"] * (180 if precision == "fp32" else 104)


def requests(n, seed=0, spacing=0.0):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        side = int(rng.choice((16, 32, 64)))
        out.append(Request(i, i * spacing, dict(nx=side, ny=side, rate=float(rng.uniform(0.001, 0.02))),
                           "fp32" if i % 2 else "fp16s"))
    return out


def test_converged_rule():
    assert converged(dict(max_ux=1.0, max_uy=0, r_u=1e-9, r_T=1, r_C=1), 1e-8, 1e-12)
    assert not converged(dict(max_ux=1.0, max_uy=0, r_u=1e-7, r_T=0, r_C=0), 1e-8, 1e-12)
    # fluid at rest: the scalar residuals decide
    assert converged(dict(max_ux=0.0, max_uy=0, r_u=1.0, r_T=1e-9, r_C=1e-10), 1e-8, 1e-12)


def test_all_requests_served_within_budget():
    reqs = requests(40, seed=1)
    budget = 3 * 64 * 64 * 180
    srv = Server(budget, max_slots=8, chunk=10, check_every=50, tol=1e-6, max_steps=3000, backend=FakeBackend)
    peak = []
    orig = srv._admit

    def admit(req, now):
        ok = orig(req, now)
        peak.append((srv.used, len(srv.active)))
        return ok
    srv._admit = admit
    results, summary = srv.run(reqs, clock=iter(range(10 ** 9)).__next__)
    assert sorted(r.id for r in results) == list(range(40))
    assert max(u for u, _ in peak) <= budget and max(n for _, n in peak) <= 8
    assert FakeSolver.live == 0 and srv.used == 0
    assert all(r.steps % 50 == 0 and r.steps <= 3000 for r in results)
    assert summary["p99_s"] >= summary["p50_s"] > 0
    for r in results:
        assert r.converged == converged(r.obs, 1e-6, 1e-12)
        assert r.converged or r.steps == 3000


def test_result_is_the_same_alone_and_in_the_mix():
    reqs = requests(12, seed=2)
    mixed = Server(10 ** 12, max_slots=16, chunk=10, check_every=50, tol=1e-6, max_steps=3000,
                   backend=FakeBackend, keep_fields=True)
    res_mix = {r.id: r for r in mixed.run(reqs, clock=iter(range(10 ** 9)).__next__)[0]}
    for req in reqs:
        alone = Server(10 ** 12, max_slots=1, chunk=10, check_every=50, tol=1e-6, max_steps=3000,
                       backend=FakeBackend, keep_fields=True)
        (r,), _ = alone.run([Request(req.id, 0.0, req.params, req.precision)],
                            clock=iter(range(10 ** 9)).__next__)
        assert r.steps == res_mix[req.id].steps
        assert r.fields == res_mix[req.id].fields


def test_oversized_request_waits_and_fifo_order():
    big = Request(0, 0.0, dict(nx=64, ny=64, rate=0.01), "fp32")
    small = Request(1, 0.0, dict(nx=16, ny=16, rate=0.5), "fp32")
    srv = Server(64 * 64 * 180, max_slots=4, chunk=10, check_every=10, tol=1e-3, max_steps=1000,
                 backend=FakeBackend)
    results, _ = srv.run([big, small], clock=iter(range(10 ** 9)).__next__)
    # the small one may not overtake the big one at admission
    adm = {r.id: r.admitted for r in results}
    assert adm[1] >= adm[0]


def test_chunk_must_divide_check_interval():
    with pytest.raises(ValueError):
        Server(1, chunk=30, check_every=100, backend=FakeBackend)


def test_node_wall_cavities_step_beside_the_batch():
    """A cavity the batch refuses (here: walls through the boundary nodes on a small lattice) is
    stepped by itself each chunk and stops at the same step as when served alone; the others,
    node-wall cavities the batch takes included, advance in the batch."""
    from paper_1708_07525_amd.lbm import node_walls
    assert node_walls(dict(sides=("nee_hot", "nee_cold", "nee_adiabatic", "nee_adiabatic")))
    assert node_walls(dict(sides=(4, 5, 6, 6)))
    assert not node_walls(dict(sides=("hot", "cold", "adiabatic", "periodic")))
    assert not node_walls(dict(nx=8))
    reqs = requests(10, seed=3)
    for r in reqs[::3]:
        r.params["sides"] = ("nee_hot", "nee_robin", "nee_adiabatic", "nee_adiabatic")
    srv = Server(10 ** 12, max_slots=16, chunk=10, check_every=50, tol=1e-6, max_steps=3000,
                 backend=FakeBackend, keep_fields=True)
    res = {r.id: r for r in srv.run(reqs, clock=iter(range(10 ** 9)).__next__)[0]}
    assert sorted(res) == list(range(10)) and FakeSolver.live == 0 and not srv.solo
    for req in reqs:
        alone = Server(10 ** 12, max_slots=1, chunk=10, check_every=50, tol=1e-6, max_steps=3000,
                       backend=FakeBackend, keep_fields=True)
        (r,), _ = alone.run([Request(req.id, 0.0, req.params, req.precision)], clock=iter(range(10 ** 9)).__next__)
        assert r.steps == res[req.id].steps and r.fields == res[req.id].fields
