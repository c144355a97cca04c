"""amgdd_solve_noalloc (for callers that cannot allocate device memory)
against amgdd_solve through the C ABI: the same iterates element by element
(FP64 bar 1e-12; the schedules and eager / graph launches give bitwise-equal
results, which is checked too) on two calls in a row, the second with a
smaller input, for plain, mixed and hybrid handles, tuned and untuned; the
static scratch bound is enforced with an error and nothing run."""

import numpy as np
import pytest

from synth import grf, make_problem
from tests.parity import rel_inf

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amgdd = pytest.importorskip("paper_1906_10575_amd.amgdd")

DEV = "cuda:0"


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device=DEV)


def _pair(p, **kw):
    s_ref = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac, **kw)
    s_na = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac, **kw)
    return s_ref, s_na


def _compare(p, s_ref, s_na, iters=3, tag=""):
    b = _t(p.b)
    x_ref = torch.zeros_like(b)
    x_na = torch.zeros_like(b)
    for k in range(iters):
        x_ref, i1, st1 = s_ref.solve(b, x_ref, rtol=0, maxit=1)
        x_na, i2, st2 = s_na.solve_noalloc(b, x_na, rtol=0, maxit=1)
        assert st1 == st2 == amgdd.OK
        err = rel_inf(x_na.cpu().numpy(), x_ref.cpu().numpy())
        print(f"[gpu-test] noalloc {tag} iteration {k + 1}: max-entry rel diff {err:.2e}, "
              f"bitwise {bool(torch.equal(x_na, x_ref))}", flush=True)
        assert err <= 1e-12
        np.testing.assert_array_equal(s_na.history(0), s_ref.history(0))
    # to tolerance: same iteration count and residual history
    x1, i1, st1 = s_ref.solve(b, torch.zeros_like(b), rtol=1e-8, maxit=100)
    x2, i2, st2 = s_na.solve_noalloc(b, torch.zeros_like(b), rtol=1e-8, maxit=100)
    assert st1 == st2 == amgdd.OK and i1.iters == i2.iters
    assert rel_inf(x2.cpu().numpy(), x1.cpu().numpy()) <= 1e-12
    hr, hn = s_ref.history(0), s_na.history(0)
    assert np.abs(hn - hr).max() <= 1e-12 * hr[0]


@pytest.mark.parametrize("kw", [dict(), dict(precision="mixed"), dict(hybrid_level=2)])
def test_noalloc_matches_solve_on_two_calls_second_smaller(kw):
    big = make_problem((20, 18, 20), (2, 2, 3), eta=2, n_fac=2, k=np.exp(grf((20, 18, 20), 1.0, 8.0, 1)))
    small = make_problem((12, 11, 10), (2, 2, 1), eta=1, n_fac=2)
    print(f"[gpu-test] noalloc {kw}: {big.n} then {small.n} rows", flush=True)
    s_ref, s_na = _pair(big, **kw)
    _compare(big, s_ref, s_na, tag=f"{kw} big")
    s_ref2, s_na2 = _pair(small, **kw)
    _compare(small, s_ref2, s_na2, tag=f"{kw} small")
    # the untuned handle stayed untuned (no tuning runs in the no-allocation call)
    assert s_na2.stats()["tail_level"] == -2 or kw.get("hybrid_level")
    # a tuned handle: the no-allocation call uses the tuned schedule
    b = _t(small.b)
    x_t, _, _ = s_ref2.solve(b, torch.zeros_like(b), rtol=0, maxit=2)
    x_n, _, _ = s_ref2.solve_noalloc(b, torch.zeros_like(b), rtol=0, maxit=2)
    assert torch.equal(x_t, x_n)


def test_noalloc_rejects_handles_beyond_the_scratch(monkeypatch):
    p = make_problem((16, 16, 16), (2, 2, 2), eta=1, n_fac=2)
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=1, n_fac=2)
    monkeypatch.setenv("AMGDD_TEST_NOALLOC_CAP", "10")   # 16 blocks + 1 problem needed
    b = _t(p.b)
    x = torch.full_like(b, 3.0)
    with pytest.raises(amgdd.AmgddError) as e:
        s.solve_noalloc(b, x, rtol=1e-8, maxit=10)
    assert e.value.status == amgdd.EUNSUPPORTED and "scratch" in str(e.value)
    assert torch.all(x == 3.0)
    monkeypatch.delenv("AMGDD_TEST_NOALLOC_CAP")
    x, info, st = s.solve_noalloc(b, torch.zeros_like(b), rtol=1e-8, maxit=50)
    assert st == amgdd.OK
    r = p.b - p.A @ x.cpu().numpy()
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(p.b)
