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
    """Energy as a function of a position x that phi carries (phi = x
    everywhere); an iteration advances x by 1, set_state restores x from phi,
    so interpolated states have fractional x."""
    M = N = 4

    def __init__(self, curve):
        self.curve = curve
        self.x = 0.0
        self.restores = 0

    def set_image(self, f, start):
        self.x = 0.0

    def energy(self):
        return float(self.curve(self.x)), (0.0, 0.0, 0.0)

    def step(self, n):
        self.x += n
        return {"iters_done": n, "converged": False}

    def phi(self):
        return torch.full((4, 4), self.x, dtype=torch.float64)

    def _empty(self, *shape):
        return torch.zeros(shape, dtype=torch.float64)

    def set_state(self, phi, w, b, k):
        self.x = float(phi[0, 0])
        self.restores += 1


@pytest.fixture()
def ws(monkeypatch):
    from paper_2003_12693_amd import warmstart
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)

    def get_state(ctx, phi, w, b):
        phi.fill_(FAKE["solver"].x)
        return int(FAKE["solver"].x)

    monkeypatch.setattr(warmstart.sr, "sr_get_state", get_state)
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


def test_smooth_acceleration_lands_in_the_window(ws):
    curve = lambda k: 1000.0 - 0.001 * k * k
    (ok, k, _, E, why), s = _run(ws, curve, 500.0)
    first = next(i for i in range(10000) if curve(i) <= 500.0 * (1 + 1e-4))
    assert ok and k == first and abs(E - 500.0) <= 500.0 * 1e-4


def test_start_below_plain_energy_is_rejected(ws):
    (ok, k, _, E, why), s = _run(ws, lambda k: 100.0 - k, 500.0)
    assert not ok and k == 0 and why == "start below the plain energy"


def test_no_progress_spends_the_budget(ws):
    (ok, k, _, E, why), s = _run(ws, lambda k: 1000.0, 500.0, k_plain=300)
    assert not ok and k == 300 and why == "budget spent"


def test_jump_over_the_window_is_resolved_between_the_last_two_iterates(ws):
    # a burst: E drops from 608 to 400 in the iteration from k = 49 to 50 (the window is 500 +- 0.05);
    # along the segment between the two iterates the energy passes through the window
    def curve(x):
        if x <= 49:
            return 1000.0 - 8.0 * x
        if x <= 50:
            return 608.0 - 208.0 * (x - 49)
        return 400.0 - 0.1 * (x - 50)
    (ok, k, _, E, why), s = _run(ws, curve, 500.0)
    assert ok and k == 50 and why == "crossing resolved on the last step"
    assert abs(E - 500.0) <= 500.0 * 1e-4
    assert 49.0 < s.x < 50.0
