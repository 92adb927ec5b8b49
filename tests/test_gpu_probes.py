"""The instrumentation kernels behind the counter and issue-class profiles: each kind runs
and computes its instruction (the literal-multiply kind bit for bit against float32
arithmetic on the CPU), and the entry points reject what their declarations exclude."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _start_values(n_blocks):
    """Each lane's eight starting values, as the kernel forms them in float32."""
    t = np.tile(np.arange(256, dtype=np.float32), n_blocks)
    a0 = t * np.float32(1e-3)
    return [a0] + [a0 + np.float32(d) for d in (0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7)]


def test_issue_probe_kinds():
    import torch
    import paper_2607_25388_amd.sgtp as sg
    n_blocks, iters = 3, 7
    for kind in range(9):
        print(f"issue probe kind {kind}", flush=True)
        out = sg.issue_probe(kind, n_blocks, iters)
        torch.cuda.synchronize()
        v = out.cpu().numpy()
        assert v.shape == (256 * n_blocks,)
        assert np.all(np.isfinite(v)), kind
        if kind == 4:
            # eight lanes' values, each multiplied by the literal 0x3f7fffef `iters` times,
            # then summed left to right
            lit = np.frombuffer(np.uint32(0x3F7FFFEF).tobytes(), np.float32)[0]
            a = _start_values(n_blocks)
            for _ in range(iters):
                a = [x * lit for x in a]
            s = a[0]
            for x in a[1:]:
                s = s + x
            assert s.dtype == np.float32
            np.testing.assert_array_equal(v, s)
    with pytest.raises(RuntimeError):
        sg.issue_probe(9, 1, 1)


def test_counter_probe_runs():
    import torch
    import paper_2607_25388_amd.sgtp as sg
    out = sg.counter_probe_fp32(4, 10)
    torch.cuda.synchronize()
    v = out.cpu().numpy()
    assert v.shape == (256,)
    assert np.all(np.isfinite(v))
