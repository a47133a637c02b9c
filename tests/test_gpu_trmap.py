"""The per-row map on the GPU at the level of single rows: hierarchical groups
of one row each (FP64 storage, K = 1, beta = 1, flat prior) make every
group's f the kernel's t(u) for u = x, and its g the kernel's r(u) x.  Each is
compared with a 40-digit decimal evaluation of the same expression."""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from gpu_helpers import DEV, Ctx, to_dev  # noqa: E402
    from paper_1310_1537_amd import glm  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


def _points(lim):
    g = np.random.default_rng(1)
    u = np.concatenate([
        np.linspace(-lim, lim, 1501),
        g.normal(0.0, 3.0, 800),
        np.exp(g.uniform(-40.0, math.log(lim), 400)) * g.choice([-1.0, 1.0], 400),
        [0.0, -0.0, 5e-324, -5e-324, 1e-300, 0.5 * math.log(2.0), -0.5 * math.log(2.0),
         math.log(1.0 + math.sqrt(2.0)), -math.log(1.0 + math.sqrt(2.0)),
         math.nextafter(math.log(1.0 + math.sqrt(2.0)), 0.0), 36.0, 37.0, -36.0, -37.0],
    ])
    return u


def _run(ctx, u, y, family):
    G = len(u)
    X = u.reshape(-1, 1).astype(np.float64)
    Xd, yd = glm.aligned_rows(to_dev(X)), to_dev(y)
    off = np.arange(G + 1, dtype=np.int64)
    gs = glm.glm_groupset_create(ctx, glm.make_desc(Xd, yd, family=family), off, tune=False)
    out = torch.empty((G, 2), dtype=torch.float64, device=DEV)
    glm.glm_logpost_grad_batched(ctx, gs, to_dev(np.ones((G, 1))), glm.make_prior(0.0), out)
    torch.cuda.synchronize()
    glm.glm_groupset_destroy(gs)
    return out.cpu().numpy()


def _ulp(v):
    return np.spacing(np.abs(v)).astype(np.float64)


@pytest.mark.parametrize("family", ["logistic", "poisson"])
def test_row_terms_to_a_few_ulps(ctx, family):
    getcontext().prec = 40
    lim = 740.0 if family == "logistic" else 700.0
    u = _points(lim)
    g = np.random.default_rng(2)
    if family == "logistic":
        y = (g.random(len(u)) < 0.5).astype(np.uint8)
        fam = glm.GLM_LOGISTIC
    else:
        y = g.integers(0, 7, len(u)).astype(np.uint8)
        fam = glm.GLM_POISSON
    got = _run(ctx, u, y, fam)
    D = Decimal
    bad = []
    for i, (ui, yi) in enumerate(zip(u, y)):
        du = D(float(ui))
        if family == "logistic":
            z = du.exp()
            # log(1 + z): the series where 1 + z would round to 1 at 40 digits
            sp = z - z * z / 2 + z * z * z / 3 if z < D("1e-12") else (D(1) + z).ln()
            t = D(int(yi)) * du - sp
            r = D(int(yi)) - D(1) / (D(1) + (-du).exp())
            # t = y u - sp rounds y u and sp before subtracting
            tol_t = 4 * (_ulp(float(t)) + _ulp(float(yi) * ui) + _ulp(float(sp)))
            tol_r = 4 * 2.0 ** -53 * (1 + abs(float(r)))
        else:
            mu = du.exp()
            t = D(int(yi)) * du - mu
            r = D(int(yi)) - mu
            tol_t = 4 * (_ulp(float(t)) + _ulp(float(yi) * ui) + _ulp(float(mu)))
            tol_r = 4 * (_ulp(float(r)) + _ulp(float(mu)) + _ulp(float(yi)))
        et = abs(got[i, 0] - float(t))
        eg = abs(got[i, 1] - float(r * du))
        if not (et <= tol_t and eg <= tol_r * abs(ui) + 4 * _ulp(float(r * du))):
            bad.append((float(ui), int(yi), got[i, 0], float(t), got[i, 1], float(r * du)))
    assert not bad, bad[:5]


def test_non_finite_u_gives_nan(ctx):
    u = np.array([np.nan, 0.5])
    got = _run(ctx, u, np.array([1, 0], np.uint8), glm.GLM_LOGISTIC)
    assert np.isnan(got[0, 0]) and np.isnan(got[0, 1])
    assert np.isfinite(got[1]).all()
