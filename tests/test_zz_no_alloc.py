"""The allocation-free field solve (pic_field_solve_noalloc) against
pic_field_solve on identical contexts, two calls in a row, the second on a
smaller grid (the library's device scratch keeps the first call's
contents)."""
import sys

import numpy as np
import pytest

from pic_cases import Case, relerr

pytestmark = pytest.mark.gpu

NAMES = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _one(case, precision, solver):
    kw = dict(solver=solver, precond_slots=4) if solver == "learned" else {}
    ref = case.gpu_sim(precision, tile=(16, 16), **kw)
    new = case.gpu_sim(precision, tile=(16, 16), **kw)
    for sim in (ref, new):
        sim.gather_push()
        sim.deposit()
    a = ref.field_solve()[0]
    b = new.field_solve_noalloc()[0]
    # the two contexts deposit J with LDS atomics in their own order, so the
    # inputs of the two solves agree to roundoff, not bit for bit
    tol = 1e-12 if precision == "fp64" else 1e-10
    assert all(abs(x - y) <= 1 for x, y in zip(a["iters"], b["iters"])), (a, b)
    assert np.allclose(a["bnorm"], b["bnorm"], rtol=1e-12, atol=0)
    for k in ("relres", "relres_recursive"):
        assert max(b[k]) <= case.rtol, k
    for n in NAMES:
        assert relerr(new.get_field(0, n), ref.get_field(0, n)) <= tol, n
    # a further step on the ordinary path from the state the variant left
    for sim in (ref, new):
        sim.step(1)
    # (FP32 particles pushed by fields that differ at roundoff can round the
    # other way: FP32-level differences in the next current)
    tol2 = 1e-11 if precision == "fp64" else 1e-5
    for n in NAMES:
        assert relerr(new.get_field(0, n), ref.get_field(0, n)) <= tol2, n
    ref.close()
    new.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_field_solve_equals_workspace_solve(precision):
    _say(f"no-alloc field solve {precision}")
    big = Case(96, 80, 2, ppc=3, gamma0=5.0, T=0.05, field_amp=0.3, seed=31, rtol=1e-12,
               maxit=400)
    small = Case(40, 24, 3, ppc=2, gamma0=5.0, T=0.05, field_amp=0.3, seed=32, rtol=1e-10,
                 maxit=400)
    _one(big, precision, "cg")
    _one(small, precision, "cg")


def test_noalloc_learned_solve():
    _say("no-alloc learned solve")
    _one(Case(64, 48, 2, ppc=2, gamma0=10.0, T=0.02, field_amp=0.2, seed=33), "fp64", "learned")


def test_noalloc_rejects_oversized_context():
    import paper_1412_2480_amd as pic
    _say("no-alloc size limit")
    case = Case(1024, 512, 1, ppc=1, gamma0=2.0, T=0.05, seed=34)   # 524288 cells > 2^18
    sim = case.gpu_sim("fp64", tile=(16, 16))
    sim.gather_push()
    sim.deposit()
    with pytest.raises(pic.PicError) as ei:
        sim.field_solve_noalloc()
    assert ei.value.code == -1 and "262144" in str(ei.value)
    sim.close()
