"""The continuous-batching loop on the GPU: every request's result is the same served alone
and served in the mix (bitwise: the batched launch runs the same per-node code and each
request is checked on its own step clock)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _requests(node_walls=False):
    from paper_1708_07525_amd.serving import Request
    rng = np.random.default_rng(12)
    out = []
    for i in range(6):
        side = int(rng.choice((32, 48, 64)))
        p = workloads.cavity_params(nx=side, ny=side, Ra=float(10 ** rng.uniform(3, 4.5)),
                                    Da=float(10 ** rng.uniform(-3, -1)), phi=float(rng.uniform(0.4, 0.9)),
                                    Le=float(rng.uniform(1, 5)), N=float(rng.uniform(-1, 1)))
        if node_walls and i % 3 == 1:
            p.update(sides=("nee_hot", "nee_robin", "nee_adiabatic", "nee_adiabatic"), Bi_T=1.0, Bi_C=2.0)
        T, C = workloads.noise_fields(side, side, (12, i))
        out.append(Request(i, 0.002 * i, p, "fp32" if i % 2 else "fp16s", None, T, C))
    return out


@pytest.mark.parametrize("node_walls", [False, True])
def test_alone_equals_mixed(node_walls):
    """With node_walls, two of the six requests have walls through the boundary nodes: the
    batch takes an FP32 one of a full two-step tile, the others are stepped beside it."""
    from paper_1708_07525_amd.serving import Request, Server
    reqs = _requests(node_walls)
    mixed = Server(10 ** 10, max_slots=8, chunk=100, check_every=500, tol=1e-6, max_steps=3000, keep_fields=True)
    res_mix, summ = mixed.run(reqs)
    mixed.close()
    assert summ["requests"] == len(reqs)
    assert summ["p99_s"] >= summ["p50_s"] > 0 and summ["aggregate_MLUPS"] > 0
    res_mix = {r.id: r for r in res_mix}
    for req in reqs:
        alone = Server(10 ** 10, max_slots=1, chunk=100, check_every=500, tol=1e-6, max_steps=3000,
                       keep_fields=True)
        (r,), _ = alone.run([Request(req.id, 0.0, req.params, req.precision, None, req.T, req.C)])
        alone.close()
        m = res_mix[req.id]
        assert r.steps == m.steps and r.converged == m.converged
        for k in ("ux", "uy", "T", "C", "rho"):
            assert np.array_equal(r.fields[k], m.fields[k]), (req.id, k)
        assert r.obs["Nu"] == m.obs["Nu"] and r.obs["Sh"] == m.obs["Sh"]


def test_budget_limits_residency():
    from paper_1708_07525_amd import footprint_bytes
    from paper_1708_07525_amd.serving import Server
    reqs = _requests()
    budget = 2 * max(footprint_bytes(r.params, r.precision) for r in reqs)
    srv = Server(budget, max_slots=8, chunk=100, check_every=500, tol=1e-6, max_steps=1000)
    seen = []
    orig = srv._admit

    def admit(req, now):
        ok = orig(req, now)
        seen.append(srv.used)
        return ok
    srv._admit = admit
    results, _ = srv.run(reqs)
    srv.close()
    assert len(results) == len(reqs) and max(seen) <= budget


def test_failed_request_is_evicted():
    """A request whose fields turn non-finite (a NaN in its initial temperature: one FP16-storage
    and one FP32 request) retires at its first check, unconverged and flagged; every other
    request's result is bitwise that of the clean mix."""
    from paper_1708_07525_amd.serving import Request, Server
    reqs = _requests()
    bad = {2, 3}
    sick = []
    for r in reqs:
        T = r.T
        if r.id in bad:
            T = r.T.copy()
            T[3, 4] = np.nan
        sick.append(Request(r.id, r.arrival, r.params, r.precision, None, T, r.C))
    runs = {}
    for name, rq in (("clean", reqs), ("sick", sick)):
        srv = Server(10 ** 10, max_slots=8, chunk=100, check_every=500, tol=1e-6, max_steps=3000, keep_fields=True)
        res, summ = srv.run(rq)
        srv.close()
        assert summ["requests"] == len(rq)
        runs[name] = {r.id: r for r in res}
    for i in bad:
        r = runs["sick"][i]
        assert r.obs["nonfinite"] and not r.converged and r.steps == 500, i
    for i, c in runs["clean"].items():
        if i in bad:
            continue
        m = runs["sick"][i]
        assert c.steps == m.steps and c.converged == m.converged, i
        for k in ("ux", "uy", "T", "C", "rho"):
            assert np.array_equal(c.fields[k], m.fields[k]), (i, k)
