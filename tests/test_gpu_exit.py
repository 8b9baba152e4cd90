"""An ordinary process that uses the library exits cleanly: a child
interpreter builds matrices (resident plan, streamed and hashed builds, whose
context keeps pinned host staging), takes sizes, trains one step and exits;
its exit status must be 0 (teardown at interpreter exit)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import numpy as np
import torch
import paper_2307_04890_amd as tn
import tn_inputs as T
n = 3000
s, d, t = T.activity_driven(n, 9000, 900, seed=1)
p = tn.Plan(n, s, d, t)
C = p.execute()
out, inn = tn.component_sizes(C, n)
C2, _ = tn.build_component_matrix_streamed(n, s, d, t, chunk_events=2000)
A = T.hash_coefficients(4, seed=2)
b, c, P, _ = tn.hash_build_proxies(n, s, d, t, A, 300)
est, lifted = tn.recombine(P, b, c, n)
params = tn.mlp_init(5)
torch.cuda.synchronize()
assert torch.equal(C, C2) and int(out.sum()) == int(inn.sum())
print("child done", int(out.sum()), int(est.sum()), flush=True)
"""


def test_child_process_exits_cleanly():
    env = dict(os.environ)
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=300)
    assert "child done" in r.stdout, r.stdout + r.stderr
    assert r.returncode == 0, (r.returncode, r.stderr[-2000:])
