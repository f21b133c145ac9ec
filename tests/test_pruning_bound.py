"""The lower bound behind the assignment's exact pruning, checked on the CPU.

For candidate k of pixel p, D of Eq. (3) is evaluated in FP32 as
  A = fl(fl(lambda dcp) + fl((1 - lambda) fl(sc / np)))      (Eq. (1))
  B = fl(1 + fl(gamma fl(sw / np)))                           (Eq. (2))
  D = fl(fl(A B) + fl(ds spw))                                (Eq. (3))
with sc >= dcp >= 0 (sums of colour distances, p itself first), sw >= 0,
lambda in [0, 1], gamma >= 0, spw >= 0.  The kernel skips the walk when
LB = fl(fl(lambda dcp) + fl(ds spw)) cannot beat the best D so far; that is
exact only if LB <= D for every such operand, which holds because FP32
rounding is monotone.  These draws cover ordinary, tiny, huge and tied
operands; numpy's float32 operations round like the kernel's.
"""
import numpy as np
import pytest

f32 = np.float32


def _d_and_lb(dcp, sc, sw, n, ds, lam, gamma, spw):
    with np.errstate(over="ignore", invalid="ignore"):
        np1 = (n + 1).astype(f32)
        qc = sc / np1
        qw = sw / np1
        A = lam * dcp + (f32(1.0) - lam) * qc
        B = f32(1.0) + gamma * qw
        D = A * B + ds * spw
        LB = lam * dcp + ds * spw
    return D, LB


def _draw(rng, size, scale):
    dcp = (rng.random(size) * scale).astype(f32)
    sc = (dcp + (rng.random(size) * scale * 40).astype(f32)).astype(f32)
    sw = (rng.random(size) * 40).astype(f32)
    n = rng.integers(0, 2000, size)
    ds = (rng.random(size) * 5000).astype(f32)
    return dcp, sc, sw, n, ds


@pytest.mark.parametrize("scale", [1e-30, 1e-6, 1.0, 1e4, 1e30])
@pytest.mark.parametrize("lam,gamma,spw", [(0.5, 64.0, 0.0961), (0.0, 64.0, 0.0961), (1.0, 0.0, 0.0961),
                                          (0.3, 7.0, 0.0), (0.5, 0.0, 0.25), (1.0, 50.0, 1e-3)])
def test_lower_bound_never_exceeds_d(scale, lam, gamma, spw):
    rng = np.random.default_rng(7)
    dcp, sc, sw, n, ds = _draw(rng, 200_000, scale)
    D, LB = _d_and_lb(dcp, sc, sw, n, ds, f32(lam), f32(gamma), f32(spw))
    finite = np.isfinite(D)
    assert finite.any()
    assert (LB[finite] <= D[finite]).all()
    # an infinite D is still >= its bound
    assert (LB[~finite & ~np.isnan(D)] <= D[~finite & ~np.isnan(D)]).all()


def test_bound_is_tight_without_path_and_contour_terms():
    """With lambda = 1 (or sc = 0) and sw = 0 the bound is D itself: ties between
    a bound and the best D really occur, which is why a tied bound is skipped
    only for a higher slot."""
    rng = np.random.default_rng(3)
    dcp, sc, sw, n, ds = _draw(rng, 10_000, 10.0)
    D, LB = _d_and_lb(dcp, sc, np.zeros_like(sw), n, ds, f32(1.0), f32(64.0), f32(0.1))
    assert (D == LB).all()
