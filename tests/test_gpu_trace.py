"""GACELLE_TRACE: a process started with it writes, at exit, one trace event
per launch of the timed kernel families (synchronous calls and server
rounds), as Chrome trace-event JSON."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import numpy as np
import oracle as orc
from paper_2511_22094_amd import lib, synth
g = lib()
d = synth.make_draw("monoexp_t2s", (2, 8, 8), 3, 0.01)
y = synth.scatter((orc.forward(d.model, d.acq, d.truth) + d.sigma * d.noise)
                  .astype(np.float32), d.mask)
m = g.Model.from_acq(d.model, d.acq)
g.gc_mcmc(m, y, d.mask, d.lb, d.ub, 2, 300, 50, 5, sigma=0.01, chunk_iters=100)
g.gc_fit_askadam(m, y, d.mask, d.lb, d.ub, n_iter=40, lam=1e-3, tv_params=(0,))
with g.Server(chunk_iters=100) as S:
    j = S.submit_mcmc(m, y, d.mask, d.lb, d.ub, 2, 300, 50, 5, sigma=0.01)
    S.wait(j)
print("child done", flush=True)
'''


def test_trace_file_lists_the_launches(tmp_path):
    path = tmp_path / "trace.json"
    env = dict(os.environ, GACELLE_TRACE=str(path), PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", CHILD], env=env, cwd=ROOT, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    ev = json.loads(path.read_text())["traceEvents"]
    names = [e["name"] for e in ev]
    # three 100-step chunks per MCMC call (direct and served), 40 Adam steps
    assert names.count("mh_chunk") == 6, names
    assert names.count("fit_step") == 40, names
    for e in ev:
        assert e["ph"] == "X" and e["dur"] > 0 and e["ts"] >= 0 and e["pid"] == 0
    # launches on one stream do not overlap
    by_stream = {}
    for e in ev:
        by_stream.setdefault(e["tid"], []).append((e["ts"], e["ts"] + e["dur"]))
    for spans in by_stream.values():
        spans.sort()
        for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
            assert b0 >= a1 - 1.0, (a0, a1, b0, b1)
