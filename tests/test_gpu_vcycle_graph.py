"""The V-cycle of the Krylov solves replayed as a captured HIP graph
(C0IP_VCYCLE_GRAPH=1, read once per process, so the solve runs in a child
process) gives the iterations and the bitwise solution of the default eager
launches, for FGMRES and flexible CG in both V-cycle precisions."""
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest
import torch

import paper_2412_05082_amd as P
from paper_2412_05082_amd.inputs import seeded_vector
from tests.gpu_util import host, say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys, json, numpy as np, torch
sys.path.insert(0, {root!r})
import paper_2412_05082_amd as P
from paper_2412_05082_amd.inputs import seeded_vector
out = {{}}
for name, dt, fcg in [("gm32", P.C0IP_F32, False), ("gm64", P.C0IP_F64, False), ("cg32", P.C0IP_F32, True)]:
    pb = P.Problem(2, 64, 3, omega=0.25, vcycle_dtype=dt)
    b = torch.from_numpy(seeded_vector(2, 3, 64, 5)).cuda()
    x = torch.zeros_like(b)
    info = pb.solve_fcg(b, x) if fcg else pb.solve(b, x)
    np.save({out!r} + name + ".npy", x.cpu().numpy())
    out[name] = info["iterations"]
    pb.close()
print(json.dumps(out))
"""


def test_graph_replay_matches_eager_launches():
    say("V-cycle graph replay vs eager")
    with tempfile.TemporaryDirectory() as d:
        prefix = os.path.join(d, "x_")
        env = dict(os.environ, C0IP_VCYCLE_GRAPH="1")
        res = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, out=prefix)], env=env,
                             capture_output=True, text=True, timeout=240)
        assert res.returncode == 0, res.stderr[-2000:]
        import json
        its = json.loads(res.stdout.strip().splitlines()[-1])
        for name, dt, fcg in [("gm32", P.C0IP_F32, False), ("gm64", P.C0IP_F64, False), ("cg32", P.C0IP_F32, True)]:
            pb = P.Problem(2, 64, 3, omega=0.25, vcycle_dtype=dt)
            b = torch.from_numpy(seeded_vector(2, 3, 64, 5)).cuda()
            x = torch.zeros_like(b)
            info = pb.solve_fcg(b, x) if fcg else pb.solve(b, x)
            pb.close()
            xg = np.load(prefix + name + ".npy")
            say(f"  {name}: eager {info['iterations']} its, graph {its[name]} its")
            assert info["iterations"] == its[name], name
            assert np.array_equal(host(x), xg), name
