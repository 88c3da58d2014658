"""The learned warm start, end to end on the GPU: the committed network
(trained on plain-solver outputs by the library's own kernels) against the
plain solve on held-out instances, and the fallback rule on degenerate
predictions."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ws():
    from paper_2003_12693_amd import warmstart
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return warmstart


def test_trained_warm_start_saves_iterations(ws):
    params = np.load(ws.WEIGHTS)
    seeds = [ws.EVAL_SEED0 + 500, ws.EVAL_SEED0 + 501]          # held out: never trained on
    summary, rows = ws.evaluate(params, seeds, log=_note)
    assert summary["accepted"] == len(seeds)
    for r in rows:
        assert r["iters_warm"] <= 0.1 * ws.K_PLAIN              # >= 90 % of the iterations saved
        assert abs(r["rel_dE"]) <= ws.E_TOL                       # the plain solve's energy, within 1e-4
        assert r["t_warm"] < r["t_plain"]


def test_degenerate_predictions_fall_back(ws):
    from paper_2003_12693_amd import cnn
    n = cnn.cnn_num_params()
    seed = [ws.EVAL_SEED0 + 502]
    p = np.zeros(n, np.float32)
    p[-1] = 1.0           # phi-hat = +CLIP everywhere: no inside, energy already below the plain solve's
    summary, rows = ws.evaluate(p, seed, k_plain=2000, log=_note)
    assert summary["accepted"] == 0 and rows[0]["reason"] == "start below the plain energy"
    assert rows[0]["cost_iters"] == 2000
    p[-1] = -1.0          # phi-hat = -CLIP everywhere: no contour, the energy cannot move
    summary, rows = ws.evaluate(p, seed, k_plain=2000, log=_note)
    assert summary["accepted"] == 0 and rows[0]["reason"] == "budget spent"
    assert rows[0]["cost_iters"] == 4000                         # both solves are charged
