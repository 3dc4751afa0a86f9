"""Differentiation form: the estimator as the backward of an autograd
Function over (positions, albedo), through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_2404_09758_amd import autograd
from paper_2404_09758_amd import scenes as S

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _setup(sc):
    o = oracle.Oracle(sc)
    tg = [o.render(sc.flat_params(True), v)[0] for v in sc.views]
    return o, tg


def _params(sc):
    pos = torch.tensor(sc.pos, device=DEV, requires_grad=True)
    alb = torch.tensor(sc.tex[0], device=DEV, requires_grad=True)
    return pos, alb


@pytest.mark.parametrize("name,pairs", [("octa", 256), ("diff", 64)])
def test_forward_loss_and_backward_match_oracle(name, pairs):
    sc = S.CONFIGS[name]()
    o, tg = _setup(sc)
    eps = [1e-3, 1e-2]
    lf = autograd.StochasticRasterLoss(sc, [torch.tensor(t, device=DEV) for t in tg], pairs, eps=eps, seed=42,
                                       device=DEV)
    pos, alb = _params(sc)
    loss = lf(pos, alb)
    ref = sum(float(o.pixel_loss(sc.flat_params(), v, t).astype(np.float64).sum()) for v, t in zip(sc.views, tg))
    assert float(loss.detach()) == pytest.approx(ref, rel=1e-12)
    loss.backward()
    Qo, Ko, _, _ = o.estimate(sc.flat_params(), sc.views, tg, 42, 1, pairs, eps)
    go = o.decode(Qo, Ko, eps, S.AVG_PAIRS, pairs)
    nv = 3 * sc.n_verts
    assert np.array_equal(pos.grad.cpu().numpy().reshape(-1), go[:nv])
    assert np.array_equal(alb.grad.cpu().numpy().reshape(-1), go[nv:])
    g = np.concatenate([pos.grad.cpu().numpy().reshape(-1), alb.grad.cpu().numpy().reshape(-1)]).astype(np.float64)
    cos = g @ go / (np.linalg.norm(g) * np.linalg.norm(go))
    assert cos >= 0.999
    # the next backward draws fresh pairs
    pos.grad = None
    lf(pos, alb).backward()
    Qo2, Ko2, _, _ = o.estimate(sc.flat_params(), sc.views, tg, 42, 2, pairs, eps)
    assert np.array_equal(pos.grad.cpu().numpy().reshape(-1), o.decode(Qo2, Ko2, eps, S.AVG_PAIRS, pairs)[:nv])


def test_backward_vs_central_finite_differences():
    """16x16 check scene, 256 pairs, central differences h = 1e-4 (Eq. 3).
    Texels: the unlit image is quadratic in them, so the estimate converges
    to the difference quotient (cosine 0.98 at 256 pairs).  Positions: a hard
    rasterizer's image error is piecewise constant in them and its difference
    quotient depends on h (h = 1e-4 vs 1e-3 agree only to cosine 0.44), so
    only a positive correlation is asserted."""
    sc = S.make_octa_small()
    o, tg = _setup(sc)
    theta = sc.flat_params()
    d = o.d
    h = 1e-4
    fd = np.zeros(d)
    for i in range(d):
        s = np.zeros(d, np.int8)
        s[i] = 1
        fp = o.pixel_loss(theta, sc.views[0], tg[0], signs_=s, sign=+1, eps=[h, h]).astype(np.float64).sum()
        fm = o.pixel_loss(theta, sc.views[0], tg[0], signs_=s, sign=-1, eps=[h, h]).astype(np.float64).sum()
        fd[i] = (fp - fm) / (2 * h)
    lf = autograd.StochasticRasterLoss(sc, [torch.tensor(t, device=DEV) for t in tg], 256, eps=(1e-3, 1e-2),
                                       seed=7, device=DEV)
    pos, alb = _params(sc)
    lf(pos, alb).backward()
    nv = 3 * sc.n_verts
    gp = pos.grad.cpu().numpy().reshape(-1).astype(np.float64)
    ga = alb.grad.cpu().numpy().reshape(-1).astype(np.float64)

    def cos(a, b):
        return a @ b / (np.linalg.norm(a) * np.linalg.norm(b))

    assert cos(ga, fd[nv:]) >= 0.97
    assert cos(gp, fd[:nv]) > 0.3


def test_diff_run_adam_lowers_loss():
    """256^2, 5120 triangles, 256^2 albedo, 64 pairs per backward: torch's
    Adam on the estimated gradients lowers the image error."""
    sc = S.make_diff_run()
    lf0 = None
    o, tg = _setup(sc)
    lf = autograd.StochasticRasterLoss(sc, [torch.tensor(t, device=DEV) for t in tg], 64, eps=(1e-3, 1e-2),
                                       seed=3, device=DEV)
    pos, alb = _params(sc)
    opt = torch.optim.Adam([{"params": [pos], "lr": 1e-3}, {"params": [alb], "lr": 1e-2}])
    losses = []
    for _ in range(30):
        opt.zero_grad()
        loss = lf(pos, alb)
        loss.backward()
        opt.step()
        losses.append(float(loss))
    del lf0
    assert losses[-1] < 0.8 * losses[0]


# ------------------------------------------------------ image-output form --

def test_render_forward_and_image_backward_match_oracle():
    """The images are the oracle's renders bit for bit; the backward of a
    downstream L1 loss (computed by torch) equals the oracle's image-form
    estimate for the same dL/dI, averaged over the pairs."""
    sc = S.make_octa_small()
    o, tg = _setup(sc)
    eps = [1e-3, 1e-2]
    pairs = 16
    rf = autograd.StochasticRender(sc, pairs, eps=eps, seed=9, device=DEV)
    pos, alb = _params(sc)
    imgs = rf(pos, alb)
    ref = np.stack([o.render(sc.flat_params(), v)[0] for v in sc.views])
    assert np.array_equal(imgs.detach().cpu().numpy(), ref)
    target = torch.tensor(np.stack(tg), device=DEV)
    w = torch.linspace(0.5, 1.5, imgs.shape[2], device=DEV)[None, None, :, None]
    loss = ((imgs - target).abs() * w).sum()
    g_img = torch.autograd.grad(loss, imgs, retain_graph=True)[0]
    loss.backward()
    Qo, Ko, _, _ = o.estimate(sc.flat_params(), sc.views, list(g_img.cpu().numpy()), 9, 1, pairs, eps,
                              image_grad=True)
    go = o.decode(Qo, Ko, eps, S.AVG_PAIRS, pairs)
    nv = 3 * sc.n_verts
    assert np.array_equal(pos.grad.cpu().numpy().reshape(-1), go[:nv])
    assert np.array_equal(alb.grad.cpu().numpy().reshape(-1), go[nv:])
    assert np.count_nonzero(go) > 0


def test_image_form_with_l2_downstream_tracks_loss_form():
    """With L = ||I - T||^2 computed downstream and frozen positions (the
    unlit colour is then linear in the albedo) the image form and the L2
    form give the same gradient up to fp32 rounding of the differences."""
    sc = S.CONFIGS["diff"]()
    _, tg = _setup(sc)
    eps = (0.0, 1e-2)
    pairs = 8
    target = torch.tensor(np.stack(tg), device=DEV)
    rf = autograd.StochasticRender(sc, pairs, eps=eps, seed=3, device=DEV)
    lf = autograd.StochasticRasterLoss(sc, [t for t in target], pairs, eps=eps, seed=3, device=DEV)
    pos, alb = _params(sc)
    ((rf(pos, alb) - target) ** 2).sum().backward()
    ga_img = alb.grad.clone()
    alb.grad = None
    lf(pos, alb).backward()
    ga_l2 = alb.grad
    assert float(ga_l2.abs().max()) > 0.1
    # per pixel the two differences differ by ~2 ulp(1) of rounding; a texel
    # sums ~16 pixels per pair: ~16 * 2.4e-7 / (2 eps) = 2e-4 per pair
    assert float((ga_img - ga_l2).abs().max()) < 2e-3
