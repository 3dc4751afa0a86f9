"""The estimator as the backward of a torch.autograd.Function.

StochasticRasterLoss(positions [V,3], albedo [H,W,3]) returns the L2 image
error f = sum_views || I(theta) - I_target ||^2 (Table 1) computed by the
HIP render; its backward is the per-pixel stochastic estimator averaged over
n_pairs antithetic pairs (Eq. 8-9, averaged by the number of pairs so that it
estimates df/dtheta).

StochasticRender(positions, albedo) returns the rendered images
[n_views, H, W, 3] themselves, so that any loss can be computed downstream
in torch; its backward receives g = dL/dI and runs the image form of the
estimator, which scatters <g_p, I+_p - I-_p> per pixel in place of the
difference of the per-pixel errors.  It estimates the vector-Jacobian
product g^T dI/dtheta and equals the L2 form (with g = 2 (I - T)) wherever
the colour is linear in the parameters.

Only theta (and the call counter that seeds the signs) is kept between
forward and backward: the perturbed renders are recomputed in the backward
pass, never stored.
"""
from __future__ import annotations

import torch

from . import api


class _EstimatorFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, positions, albedo, loss_obj):
        theta = loss_obj.pack(positions, albedo)
        loss = loss_obj.ctx.loss(theta, loss_obj.views, loss_obj.targets).sum()
        fctx.save_for_backward(theta)
        fctx.loss_obj = loss_obj
        return loss

    @staticmethod
    def backward(fctx, grad_out):
        (theta,) = fctx.saved_tensors
        lo = fctx.loss_obj
        step = lo.next_step()
        Q, K = lo.ctx.estimate_grad(theta, lo.views, lo.targets, lo.seed, step, lo.n_pairs, lo.eps)
        g = lo.ctx.decode_grad(Q, K, lo.eps, api.AVG_PAIRS, lo.n_pairs)
        lo.last_grad = g
        gp, ga = lo.split(g)
        go = grad_out.to(torch.float32)
        return go * gp, go * ga, None


class _Differentiated:
    """A scene whose positions and albedo are differentiated with the
    per-pixel stochastic estimator.  Textures beyond the albedo (normal map,
    roughness) are held fixed at their initial values.

    scene: scenes.Scene (topology, UVs, shading, views).  eps: (positions,
    albedo) perturbation magnitudes.  Each backward call draws fresh pairs
    (step counter starting at `first_step`)."""

    def __init__(self, scene, n_pairs, eps=(1e-3, 1e-2), seed=0, device=None, tuning=(16, 256, 0), first_step=1):
        self.ctx = api.Context(scene, device, tuning=tuning)
        self.device = self.ctx.device
        self.views = list(scene.views)
        self.n_pairs = int(n_pairs)
        self.seed = int(seed)
        self.n_pos = 3 * int(scene.pos.shape[0])
        self.alb_shape = tuple(scene.tex[0].shape)
        self.n_alb = int(scene.tex[0].size)
        self.fixed = [torch.as_tensor(t, dtype=torch.float32, device=self.device).reshape(-1) for t in scene.tex[1:]]
        self.eps = [float(eps[0]), float(eps[1])] + [0.0] * len(self.fixed)
        self._step = int(first_step) - 1
        self.last_grad = None

    def next_step(self):
        self._step += 1
        return self._step

    def pack(self, positions, albedo):
        for t, name in ((positions, "positions"), (albedo, "albedo")):
            if t.device != self.device or t.dtype != torch.float32:
                raise ValueError(f"{name} must be float32 on {self.device}")
        return torch.cat([positions.detach().reshape(-1), albedo.detach().reshape(-1)] + self.fixed).contiguous()

    def split(self, g):
        """The decoded gradient [d] as (positions [V,3], albedo) tensors."""
        nv = self.n_pos
        return g[:nv].view(-1, 3), g[nv:nv + self.n_alb].view(self.alb_shape)


class StochasticRasterLoss(_Differentiated):
    """L2 image loss; targets: device tensor of the views' [H,W,3] images
    concatenated (or a list of them).  Other arguments as _Differentiated."""

    def __init__(self, scene, targets, n_pairs, eps=(1e-3, 1e-2), seed=0, device=None, tuning=(16, 256, 0),
                 first_step=1):
        super().__init__(scene, n_pairs, eps=eps, seed=seed, device=device, tuning=tuning, first_step=first_step)
        if isinstance(targets, (list, tuple)):
            targets = torch.cat([t.reshape(-1) for t in targets])
        self.targets = targets

    def __call__(self, positions, albedo):
        return _EstimatorFn.apply(positions, albedo, self)


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, positions, albedo, obj):
        theta = obj.pack(positions, albedo)
        imgs = torch.stack([obj.ctx.render(theta, v, ids=False, uv=False)[0] for v in obj.views])
        fctx.save_for_backward(theta)
        fctx.obj = obj
        return imgs

    @staticmethod
    def backward(fctx, grad_out):
        (theta,) = fctx.saved_tensors
        ob = fctx.obj
        step = ob.next_step()
        g_img = grad_out.to(torch.float32).contiguous().reshape(-1)
        Q, K = ob.ctx.estimate_grad(theta, ob.views, g_img, ob.seed, step, ob.n_pairs, ob.eps, image_grad=True)
        g = ob.ctx.decode_grad(Q, K, ob.eps, api.AVG_PAIRS, ob.n_pairs)
        ob.last_grad = g
        gp, ga = ob.split(g)
        return gp, ga, None


class StochasticRender(_Differentiated):
    """The render as a differentiable function: __call__(positions, albedo)
    returns the views' images [n_views, H, W, 3] (all views must share one
    size); their backward is the image form of the estimator."""

    def __init__(self, scene, n_pairs, eps=(1e-3, 1e-2), seed=0, device=None, tuning=(16, 256, 0), first_step=1):
        super().__init__(scene, n_pairs, eps=eps, seed=seed, device=device, tuning=tuning, first_step=first_step)
        if len({(int(v.width), int(v.height)) for v in self.views}) != 1:
            raise ValueError("StochasticRender needs views of one size")

    def __call__(self, positions, albedo):
        return _RenderFn.apply(positions, albedo, self)
