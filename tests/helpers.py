"""Helpers shared by the test modules (no numerics of the method here)."""
import re
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def rel_errors(a: np.ndarray, b: np.ndarray):
    """Per-field relative L2 and Linf of a against reference b ([5, ...]).

    Density and energy use their own norms; the three momentum components
    share the norm of the whole momentum vector, so a component that is zero
    in the reference (w in a 2D flow) is not divided by zero."""
    a = a.reshape(5, -1)
    b = b.reshape(5, -1)
    l2 = np.zeros(5)
    linf = np.zeros(5)
    mom2 = np.sqrt((b[1:4] ** 2).sum())
    mominf = np.abs(b[1:4]).max()
    for m in range(5):
        d2 = np.sqrt(((a[m] - b[m]) ** 2).sum())
        dinf = np.abs(a[m] - b[m]).max()
        n2 = mom2 if 1 <= m <= 3 else np.sqrt((b[m] ** 2).sum())
        ninf = mominf if 1 <= m <= 3 else np.abs(b[m]).max()
        l2[m] = d2 / n2 if n2 > 0 else d2
        linf[m] = dinf / ninf if ninf > 0 else dinf
    return l2, linf


def header_functions():
    """Names of the functions declared in include/ocfd.h."""
    text = open(os.path.join(ROOT, "include", "ocfd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ocfd_[a-z_]+)\s*\(", text)))


def ulp_perturbed(U, seed=123):
    """U with every value moved by about one unit in the last place."""
    rng = np.random.default_rng(seed)
    return U * (1.0 + 2.2e-16 * rng.choice([-1.0, 1.0], size=U.shape))


# For smooth states the WENO7 nonlinear weights make dU/dt sensitive to
# rounding: a one-ulp change of the input moves the oracle's own dU/dt by
# ~1e-10 of its directional terms (and far more relative to near-zero net
# fields such as d rho/dt of a divergence-free flow).  Where the states are
# smooth, the GPU's dU/dt is therefore held to a multiple of that measured
# sensitivity instead of a fixed relative bound.
ROUNDOFF_FACTOR = 30.0


def assert_within_roundoff(got, ref, ref_pert, what=""):
    got = got.reshape(5, -1)
    ref = ref.reshape(5, -1)
    ref_pert = ref_pert.reshape(5, -1)
    err = np.sqrt(((got - ref) ** 2).sum(axis=1))
    noise = np.sqrt(((ref_pert - ref) ** 2).sum(axis=1))
    floor = 1e-13 * np.sqrt((ref ** 2).sum(axis=1)).max()
    print(f"{what}: |gpu - oracle| {err}, oracle one-ulp sensitivity {noise}", flush=True)
    assert np.all(err <= ROUNDOFF_FACTOR * noise + floor), (what, err / np.maximum(noise, 1e-300))
