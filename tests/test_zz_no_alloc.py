"""The allocation-free best response (sgtp_rollout_cost_noalloc, scratch in a static
device array) against sgtp_rollout_cost on the same inputs: every per-sample output and
the selection identical bit for bit, on two calls in a row, the second smaller (fewer
vehicles, fewer samples, another sweep variant), so nothing left in the shared array
by the first call leaks into the second."""

import numpy as np
import pytest

import parity as PY

pytestmark = pytest.mark.gpu

OUTPUTS = ("cost", "flags", "viol", "x_final", "noise", "choice")


def _bytes(t):
    return np.frombuffer(t.cpu().numpy().tobytes(), dtype=np.uint8)


def test_noalloc_matches_rollout_cost_on_two_calls():
    import torch
    import paper_2607_25388_amd.sgtp as sg
    planner = sg.Planner(max_agents_total=16, max_races=1)
    try:
        # large field at the entry point's largest K (throughput variant), then the
        # mid-scale race at a ragged K (two-wave variant)
        for name, agent, phase, K in (("c3", 9, 2, 65536), ("c2", 1, 1, 3000)):
            print(f"case {name} agent {agent} phase {phase} K {K}", flush=True)
            tr, race, params, _, w = PY.workload(name)
            rt = PY.build(planner, tr, race, params, K)
            ref = planner.rollout_cost(params, rt, agent, phase, want_noise=True)
            torch.cuda.synchronize()
            out = planner.rollout_cost(params, rt, agent, phase, want_noise=True, noalloc=True)
            torch.cuda.synchronize()
            for nm in OUTPUTS:
                assert np.array_equal(_bytes(out[nm]), _bytes(ref[nm])), (name, nm)
        assert planner.status() == 0
        # beyond the static array's capacity: a clear error, nothing enqueued
        tr, race, params, _, w = PY.workload("c1")
        big = PY.build(planner, tr, race, params, 65537)
        with pytest.raises(RuntimeError, match="ESHAPE"):
            planner.rollout_cost(params, big, 0, 1, noalloc=True)
    finally:
        planner.close()
