"""The autotuned schedule is cached per layout and device: a second handle
on the same workload (in this process, through the in-memory cache, and in a
fresh process, through the JSON file) skips the tuning runs and gives
bitwise-identical iterates (every schedule computes the same results)."""

import json
import os
import subprocess
import sys

import numpy as np
import pytest

from synth import grf, make_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amgdd = pytest.importorskip("paper_1906_10575_amd.amgdd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DIMS = (22, 17, 19)  # a layout no other test tunes (the in-memory cache is per process)


def _problem():
    return make_problem(DIMS, (2, 2, 2), eta=2, n_fac=2, k=np.exp(grf(DIMS, 1.0, 8.0, 1)))


def _iterates(s, b, k=3):
    x = torch.zeros_like(b)
    out = []
    for _ in range(k):
        x, info, st = s.solve(b, x, rtol=0, maxit=1)
        out.append(x.clone())
    return out


CHILD = r"""
import json, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import torch
from synth import grf, make_problem
from paper_1906_10575_amd import amgdd
d = (22, 17, 19)
p = make_problem(d, (2, 2, 2), eta=2, n_fac=2, k=np.exp(grf(d, 1.0, 8.0, 1)))
s = amgdd.Solver(p.A, p.part, p.nparts, padding=2, n_fac=2)
b = torch.as_tensor(p.b, device="cuda:0")
x, info, st = s.solve(b, rtol=0, maxit=2)
st_ = s.stats()
print(json.dumps({"cached": st_["schedule_cached"], "level": st_["tail_level"], "block": st_["tail_block"],
                  "autotune_s": st_["autotune_s"], "x": x.cpu().numpy()[:64].tolist()}))
"""


def test_second_handle_and_second_process_reuse_the_schedule(tmp_path, monkeypatch):
    path = str(tmp_path / "sched.json")
    monkeypatch.setenv("AMGDD_TUNE_CACHE", path)
    p = _problem()
    print("[gpu-test] schedule cache", p.n, flush=True)
    b = torch.as_tensor(p.b, device="cuda:0")
    s1 = amgdd.Solver(p.A, p.part, p.nparts, padding=2, n_fac=2)
    x1 = _iterates(s1, b)
    st1 = s1.stats()
    assert st1["schedule_cached"] == 0 and st1["autotune_s"] > 0 and st1["tail_level"] >= -1
    lines = [l for l in open(path).read().splitlines() if l.startswith('"')]
    assert len(lines) == 1
    assert json.loads(open(path).read())  # the file is valid JSON
    s2 = amgdd.Solver(p.A, p.part, p.nparts, padding=2, n_fac=2)
    x2 = _iterates(s2, b)
    st2 = s2.stats()
    print(f"[gpu-test]   tuned {st1['autotune_s']:.3f} s -> cached {st2['autotune_s'] * 1e3:.2f} ms, schedule "
          f"({st2['tail_level']}, {st2['tail_block']})", flush=True)
    assert st2["schedule_cached"] == 1 and st2["autotune_s"] < 0.05
    assert (st2["tail_level"], st2["tail_block"]) == (st1["tail_level"], st1["tail_block"])
    for a, c in zip(x1, x2):
        assert torch.equal(a, c)
    # a fresh process reads the file
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], capture_output=True, text=True, timeout=240,
                       env=dict(os.environ, AMGDD_TUNE_CACHE=path))
    assert r.returncode == 0, r.stderr[-2000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["cached"] == 1 and (out["level"], out["block"]) == (st1["tail_level"], st1["tail_block"])
    np.testing.assert_array_equal(np.array(out["x"]), x1[1].cpu().numpy()[:64])
    # a different layout (padding 1) is a different key: tuned again
    s3 = amgdd.Solver(p.A, p.part, p.nparts, padding=1, n_fac=2)
    s3.solve(b, rtol=0, maxit=1)
    assert s3.stats()["schedule_cached"] == 0
    assert len([l for l in open(path).read().splitlines() if l.startswith('"')]) == 2
