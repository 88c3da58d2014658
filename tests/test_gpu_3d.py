"""GPU parity of the 3-D solver (include/sr3d.h) against the 3-D oracle:
the edge map, one outer iteration from identical states (teacher forcing)
on cubic and non-cubic volumes and parameter sets, a short trajectory from
set_image, and the per-kernel profile counts."""
import numpy as np
import pytest

from oracle import sr_oracle as O
from oracle import sr_oracle3d as O3
from paper_2003_12693_amd import synth

from tests.helpers import as64, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# the paper's 3-D (mandible) weights, with a 5 x 5 x 5 window
MANDIBLE = dict(gamma=5.0, alpha=4.0, beta=0.2, mu=3.0, tau=0.05, eps=1.0, band_l=1.0, d=4.0, R=2, S=5,
                sigma=1.5, rho=1000.0, s_exp=2, tol_inner=0.0, zero_tol=1e-3)


def _note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def sr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_12693_amd import sr as srmod
    srmod.load()
    return srmod


def _cuda(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.float32))).cuda()


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _params(sr, **kw):
    return sr.sr_params_default(**dict(MANDIBLE, **kw))


def _oparams(**kw):
    d = dict(MANDIBLE, **kw)
    return O.Params(**{k: v for k, v in d.items() if k in O.Params.__dataclass_fields__})


@pytest.mark.parametrize("shape", [(8, 8, 8), (16, 32, 8), (32, 16, 64)])
def test_edge_map_3d(sr, shape):
    _note(f"3-D edge map {shape}")
    f, phi0 = synth.balls3d(*shape, seed=11)
    s = sr.Solver3D(*shape, _params(sr))
    s.set_image(_cuda(f), _cuda(phi0))
    phi, w, b, g = s.get_state()
    ref = O3.edge_map(as64(f), 1.5, 1000.0, 2)
    np.testing.assert_allclose(_np(g), ref, atol=2e-5, rtol=1e-4)
    np.testing.assert_array_equal(_np(phi), as64(phi0))
    gw = O3.grad_fwd(as64(phi0))
    for c in range(3):
        np.testing.assert_allclose(_np(w[c]), gw[c], atol=1e-5)
    assert np.all(_np(b) == 0)


def _check_w_b(ref, gw, gb):
    nref = np.sqrt(sum(c ** 2 for c in ref.w))
    ngpu = np.sqrt(sum(c ** 2 for c in gw))
    flips = (ngpu > 0.5) != (nref > 0.5)
    assert flips.mean() <= 1e-3, flips.mean()
    ok = ~flips
    for c in range(3):
        d = np.abs(gw[c][ok] - ref.w[c][ok])
        assert np.count_nonzero(d > 2e-3) <= max(2, 1e-5 * d.size) and d.max() <= 2e-2, d.max()
        np.testing.assert_allclose(gb[c][ok], ref.b[c][ok], atol=2e-3 * (1 + np.abs(ref.b[c][ok]).max()))


@pytest.mark.parametrize("shape,kw,k", [((32, 32, 32), {}, 0), ((32, 32, 32), {}, 3),
                                        ((16, 32, 64), dict(R=1, d=2.0, S=3), 2),
                                        ((64, 8, 16), dict(gamma=4.0, mu=8.0, tau=0.1, S=3, R=3, d=5.0), 2),
                                        ((8, 8, 8), {}, 1)])
def test_teacher_forced_3d(sr, shape, kw, k):
    """One outer iteration from the (FP32-rounded) oracle state after k
    iterations: phi within 1e-5 relative L2, w and b gate-flip-aware."""
    _note(f"3-D teacher forced {shape} {kw} k={k}")
    f, phi0 = synth.balls3d(*shape, seed=sum(shape))
    P = _oparams(**kw)
    st, g = O3.solve(as64(f), as64(phi0), P, k)
    st = O3.State(as64(st.phi), tuple(as64(c) for c in st.w), tuple(as64(c) for c in st.b), k)
    ref, _ = O3.sb_iteration(st, g, P)
    s = sr.Solver3D(*shape, _params(sr, **kw))
    s.set_image(_cuda(f), _cuda(phi0))
    s.set_state(_cuda(st.phi), _cuda(np.stack(st.w)), _cuda(np.stack(st.b)), k)
    assert s.step(1) == k + 1
    phi, w, b, _ = s.get_state()
    assert rel_l2(_np(phi), ref.phi) <= 1e-5
    _check_w_b(ref, _np(w), _np(b))


def test_short_trajectory_3d(sr):
    """5 iterations from set_image on both sides."""
    _note("3-D trajectory")
    shape = (32, 32, 32)
    f, phi0 = synth.balls3d(*shape, seed=5)
    P = _oparams()
    st, g = O3.solve(as64(f), as64(phi0), P, 5)
    s = sr.Solver3D(*shape, _params(sr))
    s.set_image(_cuda(f), _cuda(phi0))
    assert s.step(5) == 5
    phi, _, _, _ = s.get_state()
    assert rel_l2(_np(phi), st.phi) <= 1e-4


def test_profile_counts_3d(sr):
    shape = (16, 16, 16)
    f, phi0 = synth.balls3d(*shape, seed=9)
    s = sr.Solver3D(*shape, _params(sr, S=2))
    s.set_image(_cuda(f), _cuda(phi0))
    prof = sr.sr3_profile(s.ctx, 3)
    assert prof["window"][1] == 3 * 3 * 3 and prof["rhs"][1] == 3 * 2
    assert prof["fft"][1] == 3 * 2 * 5 and prof["w_step"][1] == 3
    assert all(v[0] > 0 for v in prof.values())
    assert s.step(1) == 4
