"""What the trained warm-start network gains over plain PGS.

The network is trained end to end on the GPU by the library's own kernels:
tight plain runs of drop scenes (seeds 1000+) are logged, the network is fit
with Adam, and held-out drop scenes (seeds 2000+) are stepped at contact
residual 1e-4 (cap 200 sweeps) with a cold start (plain PGS), the classic
previous-impulse start and the learned start.  The learned start must cut
the mean sweeps per scene and the wall time per step against plain PGS, each
with a 95% confidence interval of the paired difference that excludes zero;
every step it reports as solved must meet the tolerance.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL, CAP, STEPS = 1e-4, 200, 240


@pytest.fixture(scope="module")
def trained():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_14405_amd import train as T
    x, t = T.log_dataset(n_scenes=512, seed0=1000, steps=STEPS)
    assert x.shape[0] > 10000
    net = T.fit(x, t, epochs=100, lr=1e-3, seed=0)
    return T, net


def ci95(d):
    d = np.asarray(d, np.float64)
    return d.mean(), 1.96 * d.std(ddof=1) / np.sqrt(d.size)


def test_learned_gain_over_plain_pgs(trained):
    from paper_2106_14405_amd import _lib as L
    T, net = trained
    n = 4096
    cold = T.evaluate(L.COLD, None, n_scenes=n, seed0=2000, steps=STEPS, tol=TOL, cap=CAP)
    prev = T.evaluate(L.PREV, None, n_scenes=n, seed0=2000, steps=STEPS, tol=TOL, cap=CAP)
    lrn = T.evaluate(L.LEARNED, net, n_scenes=n, seed0=2000, steps=STEPS, tol=TOL, cap=CAP)
    s_c, s_p, s_l = (T.summary(r) for r in (cold, prev, lrn))
    print("\ncold   ", s_c, "\nprev   ", s_p, "\nlearned", s_l)
    # sweeps: per scene, mean over its steps with contacts; paired over scenes
    act = cold["contacts"] > 0
    assert np.array_equal(act[:30], lrn["contacts"][:30] > 0)  # same trajectories before any contact
    per_c = np.array([cold["sweeps"][:, s][act[:, s]].mean() for s in range(n) if act[:, s].any()])
    act_l = lrn["contacts"] > 0
    per_l = np.array([lrn["sweeps"][:, s][act_l[:, s]].mean() for s in range(n) if act[:, s].any()])
    m, h = ci95(per_l - per_c)
    print(f"sweeps learned - cold per scene: {m:.2f} +- {h:.2f}")
    assert m + h < 0
    # wall time: paired over the steps that have contacts
    steps = np.nonzero(act.any(axis=1))[0]
    m, h = ci95(lrn["ms"][steps] - cold["ms"][steps])
    print(f"ms/step learned - cold: {m:.3f} +- {h:.3f} (cold {cold['ms'][steps].mean():.3f})")
    assert m + h < 0
    # a step reported as solved meets the tolerance
    ok = (lrn["flags"] & L.FLAG_NOT_CONVERGED) == 0
    assert np.all(lrn["residual"][ok & act_l] <= TOL)
    # and the learned start never does worse than the classic one by much
    assert s_l["mean"] <= 1.05 * s_p["mean"]
