"""Shared test helpers: parameter sets for both sides and dtype plumbing.

The oracle and the HIP library each get their parameters from the same
plain dict here; neither imports the other.
"""
import numpy as np

from oracle import sr_oracle as O

# The paper's two-circles parameters with the per-workload eps / R / sigma.
PAPER_FIG1 = dict(gamma=4.0, alpha=4.0, beta=0.2, mu=8.0, tau=0.1, eps=1.5, band_l=1.0, d=5.0,
                  R=3, sigma=1.5, rho=1000.0, s_exp=2, S=3, tol_inner=0.0, zero_tol=1e-3)


def oracle_params(**kw):
    d = dict(PAPER_FIG1)
    d.update({k: v for k, v in kw.items() if k in O.Params.__dataclass_fields__})
    return O.Params(**d)


def gpu_params(**kw):
    from paper_2003_12693_amd import sr
    d = dict(PAPER_FIG1)
    d.update(kw)
    return sr.sr_params_default(**d)


def f32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float32))


def as64(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
