"""The optimiser of Sec. 5 on the mid configuration: 100 Adam steps of the
per-pixel estimator (Eq. 8, count-averaged, 16 pairs over 8 ring views of a
20480-triangle icosphere, 512^2 Lambert renders, lr 1e-3) lower the L2
image error of Table 1 against the target renders.  Run through the C ABI
(dr_estimate_grad, dr_step, dr_loss) in the batched launch shape."""
import numpy as np
import pytest
import torch

from paper_2404_09758_amd import api
from paper_2404_09758_amd import scenes as S

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def test_mid_config_adam_lowers_the_l2_error_over_100_steps():
    sc = S.make_mid()
    ctx = api.Context(sc, DEV, tuning=(16, 256, 0))
    th = torch.tensor(sc.flat_params(), device=DEV)
    tt = torch.tensor(sc.flat_params(True), device=DEV)
    tg = torch.cat([ctx.render(tt, v, ids=False, uv=False)[0].reshape(-1) for v in sc.views])
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    Q, K = ctx.new_accumulators()
    losses = [float(ctx.loss(th, sc.views, tg).sum())]
    for t in range(1, sc.steps + 1):
        ctx.estimate_grad(th, sc.views, tg, sc.seed, t, sc.n_pairs, sc.eps, Q=Q, K=K)
        ctx.step(th, m, v, t, Q, K, sc.eps, sc.n_pairs, kind=api.ADAM, averaging=api.AVG_COUNT, lr=sc.lr)
        if t % 25 == 0:
            losses.append(float(ctx.loss(th, sc.views, tg).sum()))
    torch.cuda.synchronize()
    print("[convergence] mid L2 at steps 0, 25, 50, 75, 100:", [f"{x:.1f}" for x in losses], flush=True)
    assert all(np.isfinite(losses))
    # every quarter of the run lowers the error, and the run as a whole by a third or more
    assert all(b < a for a, b in zip(losses, losses[1:])), losses
    assert losses[-1] < 0.67 * losses[0], losses
    st = ctx.stats()
    assert st["nonfinite"] == 0
