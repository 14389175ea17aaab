"""The allocation-free entry point (flood_filtration_noalloc, static device
scratch) against flood_filtration with a caller workspace, through the C
ABI: two calls in a row, the second on a smaller problem, so the second
runs over the first one's leftovers in the shared scratch."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from paper_2509_22432_amd import _lib, api

from gpu_helpers import run_single

pytestmark = pytest.mark.gpu


def _outputs(run):
    return ([t.cpu().numpy() for t in run.f], [t.cpu().numpy() for t in run.win_x],
            [t.cpu().numpy() for t in run.win_a])


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_equals_workspace_call(order):
    cases = [(synth.config_cloud(2, 300_000), 1500, 6), (synth.config_cloud(1), 64, 4)]
    for X, n_lm, k in cases:
        res = run_single(X, n_lm, k)
        pb = res["pb"]
        ws_bytes = _lib.lib().flood_filtration_workspace_size(ctypes.byref(pb.struct()), None)
        assert 0 < ws_bytes <= 64 << 20, ws_bytes
        print("noalloc: N", len(X), "L", n_lm, "k", k, "workspace", ws_bytes, flush=True)
        ref = _outputs(res["run"])
        run = api.FloodRun(pb, None, count_evals=True, noalloc=True)
        assert run.ws is None
        run()
        torch.cuda.synchronize()
        got = _outputs(run)
        for part in range(3):
            for d in range(4):
                assert np.array_equal(got[part][d], ref[part][d]), (len(X), part, d)
        assert int(run.evals.item()) > 0
