"""GPU: the sliced-ELL layout options through the C ABI — 16-bit or int32
column indices (AMGDD_INDEX32), rows of grouped levels sorted by length or
kept in local order (AMGDD_SORT_WINDOW=0), paired or unpaired load steps
(AMGDD_UNPAIRED).

Index width and row order change neither the entries of a row nor the order
in which each lane adds them (padding adds exact zeros), so every iterate is
bitwise identical, for AMG-DD, the V-cycle and the hybrid cycle, in FP64 and
in mixed precision.  Unpaired steps give the lanes of a grouped row other
subsets of its entries, so their iterates are held to the oracle bar
instead (1e-12 relative, FP64)."""

import sys

import numpy as np
import pytest

from oracle import amg, composite, cycles
from synth import config, grf, make_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amgdd = pytest.importorskip("paper_1906_10575_amd.amgdd")

DEV = "cuda:0"
ENV = ("AMGDD_INDEX32", "AMGDD_SORT_WINDOW", "AMGDD_UNPAIRED")

CASES = {
    "3d_20_var_eta2": lambda: make_problem((20, 18, 20), (2, 2, 3), eta=2, n_fac=2,
                                           k=np.exp(grf((20, 18, 20), 1.0, 8.0, 1))),
    "3d_30_ragged_4x4x4": lambda: make_problem((30, 30, 30), (4, 4, 4), eta=1, n_fac=2),
    "p2_aniso_72": lambda: config("p2", scale=72),
}


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device=DEV)


def _run(p, monkeypatch, env, precision="fp64", hybrid=0, iters=4):
    for k in ENV:
        monkeypatch.delenv(k, raising=False)
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac, precision=precision, hybrid_level=hybrid)
    b = _t(p.b)
    x, info, st = s.solve(b, rtol=0, maxit=iters)
    assert st == amgdd.OK and info.iters == iters
    xv, _, stv = s.vsolve(b, rtol=0, maxit=iters)
    assert stv == amgdd.OK
    out = (x.cpu().numpy(), xv.cpu().numpy())
    s.close()
    for k in ENV:
        monkeypatch.delenv(k, raising=False)
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_index_width_and_row_order_are_bitwise_neutral(name, precision, monkeypatch):
    p = CASES[name]()
    say("layout neutrality", name, precision, p.n)
    ref = _run(p, monkeypatch, {}, precision)
    for env in ({"AMGDD_INDEX32": "1"}, {"AMGDD_SORT_WINDOW": "0"}, {"AMGDD_SORT_WINDOW": "32"},
                {"AMGDD_INDEX32": "1", "AMGDD_SORT_WINDOW": "0"}):
        got = _run(p, monkeypatch, env, precision)
        say("  ", env)
        assert np.array_equal(got[0], ref[0]), env
        assert np.array_equal(got[1], ref[1]), env


def test_hybrid_cycle_is_bitwise_neutral_to_row_order_and_index_width(monkeypatch):
    p = CASES["3d_30_ragged_4x4x4"]()
    say("hybrid layout neutrality", p.n)
    ref = _run(p, monkeypatch, {}, hybrid=2)
    for env in ({"AMGDD_INDEX32": "1"}, {"AMGDD_SORT_WINDOW": "0"}):
        got = _run(p, monkeypatch, env, hybrid=2)
        assert np.array_equal(got[0], ref[0]), env


@pytest.mark.parametrize("name", list(CASES))
def test_unpaired_steps_match_the_oracle(name, monkeypatch):
    p = CASES[name]()
    say("unpaired steps vs oracle", name, p.n)
    H = amg.setup(p.A)
    comps = composite.build_all(H, p.part, p.nparts, p.eta)
    coarse = cycles.CoarseSolver(H.A[H.L])
    for env in ({"AMGDD_UNPAIRED": "1"}, {"AMGDD_UNPAIRED": "1", "AMGDD_INDEX32": "1"}):
        x, xv = _run(p, monkeypatch, env, iters=3)
        xo = np.zeros(p.n)
        xvo = np.zeros(p.n)
        for _ in range(3):
            xo = cycles.amgdd_iteration(H, comps, p.b, xo, p.n_fac, coarse)
            xvo = cycles.vcycle(H, xvo, p.b, coarse=coarse)
        err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
        errv = np.linalg.norm(xv - xvo) / np.linalg.norm(xvo)
        say("  ", env, f"amgdd {err:.2e} vcycle {errv:.2e}")
        assert err <= 1e-12 and errv <= 1e-12, (env, err, errv)
