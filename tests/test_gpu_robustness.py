"""Failure paths and restarts on the device, forced from the host (no kernel
is made to fault): an allocation cap that makes setup fail with ENOMEM and
leaves the library usable, and a resumed solve (10 iterations = 5 + 5,
bitwise) — between outer iterations the iterate is the whole state."""

import os
import sys

import numpy as np
import pytest

from synth import make_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amgdd = pytest.importorskip("paper_1906_10575_amd.amgdd")


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("hybrid_level", [0, 2])
def test_resume_is_bitwise(hybrid_level):
    p = make_problem((20, 18, 20), (2, 2, 3), eta=2, n_fac=2)
    say("resume", p.n, "hybrid", hybrid_level)
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac, hybrid_level=hybrid_level)
    b = torch.as_tensor(p.b, device="cuda:0")
    x10, _, _ = s.solve(b, rtol=0, maxit=10)
    x5, _, _ = s.solve(b, rtol=0, maxit=5)
    x55, info, st = s.solve(b, x5, rtol=0, maxit=5)
    assert st == amgdd.OK and info.iters == 5
    assert torch.equal(x10, x55)
    xv10, _, _ = s.vsolve(b, rtol=0, maxit=10)
    xv5, _, _ = s.vsolve(b, rtol=0, maxit=5)
    xv55, _, _ = s.vsolve(b, xv5, rtol=0, maxit=5)
    assert torch.equal(xv10, xv55)


def test_allocation_cap_gives_enomem_and_recovers(monkeypatch):
    p = make_problem((24, 24, 24), (2, 2, 2), eta=1, n_fac=2)
    say("allocation cap", p.n)
    monkeypatch.setenv("AMGDD_TEST_MAX_BYTES", str(1 << 20))
    with pytest.raises(amgdd.AmgddError) as e:
        amgdd.Solver(p.A, p.part, p.nparts, padding=1)
    assert e.value.status == amgdd.ENOMEM
    monkeypatch.delenv("AMGDD_TEST_MAX_BYTES")
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=1)
    b = torch.as_tensor(p.b, device="cuda:0")
    x, info, st = s.solve(b, rtol=1e-8, maxit=100)
    assert st == amgdd.OK
    r = p.b - p.A @ x.cpu().numpy()
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(p.b)
    # a failing solve (non-finite right-hand side) leaves the handle usable and
    # destroyable
    bad = b.clone()
    bad[3] = float("nan")
    with pytest.raises(amgdd.AmgddError) as e2:
        s.solve(bad, rtol=1e-8, maxit=5)
    assert e2.value.status == amgdd.EBREAKDOWN
    x2, _, st3 = s.solve(b, rtol=1e-8, maxit=100)
    assert st3 == amgdd.OK and torch.equal(x, x2)
    s.close()


def test_trace_ranges_do_not_change_results(tmp_path):
    # AMGDD_TRACE=1 wraps setup, autotuning, capture, solves and iterations
    # in roctx ranges; a child process solves with tracing on and must give
    # the same iterate as this one with tracing off
    import subprocess
    p = make_problem((16, 16, 16), (2, 2, 2), eta=1, n_fac=2)
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=1, n_fac=2)
    x, _, _ = s.solve(torch.as_tensor(p.b, device="cuda:0"), rtol=0, maxit=4)
    out = tmp_path / "x.npy"
    code = (
        "import numpy as np, torch\n"
        "from paper_1906_10575_amd import amgdd\n"
        "from synth import make_problem\n"
        "p = make_problem((16, 16, 16), (2, 2, 2), eta=1, n_fac=2)\n"
        "s = amgdd.Solver(p.A, p.part, p.nparts, padding=1, n_fac=2)\n"
        "x, _, _ = s.solve(torch.as_tensor(p.b, device='cuda:0'), rtol=0, maxit=4)\n"
        f"np.save({str(out)!r}, x.cpu().numpy())\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, AMGDD_TRACE="1", PYTHONPATH=root)
    r = subprocess.run([sys.executable, "-c", code], env=env, cwd=root, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    assert np.array_equal(np.load(out), x.cpu().numpy())
