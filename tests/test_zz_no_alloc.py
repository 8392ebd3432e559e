"""lbm_observables_static (no device allocation: the library's fixed scratch) against
lbm_observables, through the C ABI: two identical contexts advanced the same way, one observed
with each entry point, give the same observables and fields bit for bit; two calls in a row,
the second on a smaller lattice; lattices beyond the scratch limits are refused."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _pair(nx, ny, prec, seed):
    from paper_1708_07525_amd import Solver
    case = workloads.grf_cavity(seed=seed, n=max(nx, ny))
    p = dict(case["params"], nx=nx, ny=ny)
    kw = dict(phi=case["phi"][:ny, :nx], T=case["T"][:ny, :nx], C=case["C"][:ny, :nx])
    return Solver(p, precision=prec, **kw), Solver(p, precision=prec, **kw)


def _same(a, b):
    for k in ("step", "Nu", "Sh", "mass", "heat", "solute", "max_ux", "max_uy", "r_u", "r_T", "r_C", "nonfinite",
              "status"):
        assert a[k] == b[k], (k, a[k], b[k])


@pytest.mark.parametrize("prec", ["fp32", "fp64", "fp16s"])
def test_static_observables_match_the_allocating_call(prec):
    for nx, ny in ((256, 200), (96, 67)):          # the second call on a smaller lattice
        print(f"case {prec} {nx}x{ny}", flush=True)
        a, b = _pair(nx, ny, prec, seed=3)
        for steps, fields in ((150, True), (50, False), (30, True)):
            a.step(steps)
            b.step(steps)
            oa = a.observables(fields=fields, static=True)
            ob = b.observables(fields=fields)
            _same(oa, ob)
            if fields:
                for k in ("rho", "ux", "uy", "T", "C"):
                    assert np.array_equal(oa["fields"][k], ob["fields"][k]), k
        a.close()
        b.close()


def test_static_observables_refuse_lattices_beyond_the_scratch():
    from paper_1708_07525_amd import Solver
    from paper_1708_07525_amd.lbm import EINVAL, LbmError
    tall = Solver(workloads.cavity_params(nx=3, ny=16385), T=0.5, C=0.5, precision="fp32")
    with pytest.raises(LbmError) as ei:
        tall.observables(static=True)
    assert ei.value.status == EINVAL
    tall.observables()                              # the allocating call still serves it
    tall.close()
    big = Solver(workloads.cavity_params(nx=1100, ny=1000), T=0.5, C=0.5, precision="fp32")
    big.step(4)
    big.observables(static=True)                    # observables alone fit
    with pytest.raises(LbmError) as ei:
        big.observables(fields=True, static=True)   # 1.1M nodes of fields do not
    assert ei.value.status == EINVAL
    big.close()
