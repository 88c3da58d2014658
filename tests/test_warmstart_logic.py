"""Host-side decision logic of the warm start (no GPU): acceptance at the
energy crossing, undo of an over-long chunk, rejection of a start below the
plain energy, and the budget fallback, driven by a fake solver whose energy
follows a scripted curve E(k)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


class FakeNet:
    def forward(self, f, g, phi0, clip):
        return torch.zeros((1, 4, 4))


class FakeSolver:
    """Energy as a function of the iteration count; snapshots are (k,)."""
    M = N = 4

    def __init__(self, curve):
        self.curve = curve
        self.k = 0
        self.restores = 0

    def set_image(self, f, start):
        self.k = 0

    def energy(self):
        return float(self.curve(self.k)), (0.0, 0.0, 0.0)

    def step(self, n):
        self.k += n
        return {"iters_done": n, "converged": False}

    def _empty(self, *shape):
        return torch.zeros(shape)

    def set_state(self, phi, w, b, k):
        self.k = int(k)
        self.restores += 1


@pytest.fixture()
def ws(monkeypatch):
    from paper_2003_12693_amd import warmstart
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    monkeypatch.setattr(warmstart.sr, "sr_get_state", lambda ctx, phi, w, b: FAKE["solver"].k)
    return warmstart


FAKE = {}


def _run(ws, curve, E_plain, k_plain=10000):
    s = FakeSolver(curve)
    s.ctx = None
    FAKE["solver"] = s
    z = torch.zeros((4, 4))
    return ws.warm_solve(s, FakeNet(), z, z, z, k_plain, E_plain), s


def test_accepts_at_the_crossing(ws):
    # steady descent of 1 per iteration from 1000: the window |E - 500| <= 0.05 holds only at k = 500
    (ok, k, _, E, why), s = _run(ws, lambda k: 1000.0 - k, 500.0)
    assert ok and k == 500 and E == 500.0 and why == "energy reached"


def test_overlong_chunk_is_undone(ws):
    # the descent steepens 20x at k = 400: a chunk sized from the slow rate jumps far below the
    # window, is undone from the snapshot and retried shorter until the run stops at E(405) = 500
    curve = lambda k: 1000.0 - k if k < 400 else 600.0 - 20.0 * (k - 400)
    (ok, k, _, E, why), s = _run(ws, curve, 500.0)
    assert s.restores >= 1
    assert ok and k == 405 and E == 500.0 and why == "energy reached"


def test_smooth_acceleration_resolves_the_crossing_to_one_iteration(ws):
    curve = lambda k: 1000.0 - 0.001 * k * k
    (ok, k, _, E, why), s = _run(ws, curve, 500.0)
    first = next(i for i in range(10000) if curve(i) <= 500.0 * (1 + 1e-4))
    assert ok and k == first


def test_start_below_plain_energy_is_rejected(ws):
    (ok, k, _, E, why), s = _run(ws, lambda k: 100.0 - k, 500.0)
    assert not ok and k == 0 and why == "start below the plain energy"


def test_no_progress_spends_the_budget(ws):
    (ok, k, _, E, why), s = _run(ws, lambda k: 1000.0, 500.0, k_plain=300)
    assert not ok and k == 300 and why == "budget spent"


def test_jump_over_the_window_in_one_iteration_is_accepted_there(ws):
    # a burst: E drops from 600 to 400 between k = 49 and 50 (the window is 500 +- 0.05)
    curve = lambda k: 1000.0 - 8.0 * k if k < 50 else 400.0 - 0.1 * (k - 50)
    (ok, k, _, E, why), s = _run(ws, curve, 500.0)
    assert ok and k == 50 and why == "crossed within one iteration"
