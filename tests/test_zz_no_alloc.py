"""The allocation-free estimate (dr_estimate_grad_noalloc) against
dr_estimate_grad, through the C ABI.

The allocation-free call takes its scratch from the library's static
device array; its Q and K must equal those of dr_estimate_grad bit for bit
(Eq. 8 summed over pairs and views).  Two calls in a row share the array,
the second on a smaller input, so a stale bin counter or group sum left by
the first call would show in the second.  A call whose scratch exceeds the
array is refused on the host and leaves Q and K untouched.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from paper_2404_09758_amd import _lib as L
from paper_2404_09758_amd import api
from paper_2404_09758_amd import scenes as S
from tests import helpers as H

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def targets(sc):
    o = oracle.Oracle(sc)
    th = sc.flat_params(True)
    return dev(np.concatenate([o.render(th, v)[0].reshape(-1) for v in sc.views]))


def both(sc, tuning, pairs, seed, step):
    """(Q, K) of dr_estimate_grad and of dr_estimate_grad_noalloc on the
    same inputs, each into fresh accumulators."""
    ctx = api.Context(sc, DEV, tuning=tuning)
    ctx.set_adaptive_bins(False)
    theta = dev(sc.flat_params())
    tg = targets(sc)
    out = []
    for noalloc in (False, True):
        Q, K = ctx.new_accumulators()
        ctx.estimate_grad(theta, sc.views, tg, seed, step, pairs, sc.eps, Q, K, noalloc=noalloc)
        out.append((host(Q), host(K)))
    st = ctx.stats()
    return out, st


def large_scene():
    return H.sphere_scene(6, 0, res=(96, 80), shading=S.SHADING_LAMBERT, tex_shapes=((48, 48, 3),), seed=1,
                          views=2)


def small_scene():
    return S.make_tiny()


def subdiv_scene():
    sc = H.sphere_scene(1, 0, res=(72, 64), shading=S.SHADING_UNLIT, tex_shapes=((32, 32, 3),), seed=7, views=1)
    sc.subdiv_levels = 2
    return sc


@pytest.mark.parametrize("tuning", [(16, 256, 0), (8, 1, 1), (32, 64, 3)])
def test_noalloc_equals_estimate_twice_second_smaller(tuning):
    print(f"[noalloc] tuning {tuning}: large scene, 5 pairs x 2 views", flush=True)
    (ref, got), st = both(large_scene(), tuning, 5, 21, 3)
    assert np.array_equal(ref[0], got[0]), "Q differs (first call)"
    assert np.array_equal(ref[1], got[1]), "K differs (first call)"
    assert np.abs(ref[0]).sum() > 0 and ref[1].sum() > 0
    print(f"[noalloc] tuning {tuning}: tiny scene, 1 pair x 1 view", flush=True)
    (ref, got), _ = both(small_scene(), tuning, 1, 22, 4)
    assert np.array_equal(ref[0], got[0]), "Q differs (second, smaller call)"
    assert np.array_equal(ref[1], got[1]), "K differs (second, smaller call)"
    assert ref[1].sum() > 0


def test_noalloc_matches_oracle_and_subdivision():
    """The allocation-free call on the tiny scene equals the oracle; on a
    subdivision surface (its tessellated positions also come from the
    array) it equals dr_estimate_grad."""
    sc = small_scene()
    o = oracle.Oracle(sc)
    tg = o.render(sc.flat_params(True), sc.views[0])[0]
    Qo, Ko, _, _ = o.estimate(sc.flat_params(), sc.views, [tg], 17, 2, 3, sc.eps)
    ctx = api.Context(sc, DEV)
    Q, K = ctx.new_accumulators()
    ctx.estimate_grad(dev(sc.flat_params()), sc.views, dev(tg.reshape(-1)), 17, 2, 3, sc.eps, Q, K, noalloc=True)
    assert np.array_equal(host(Q), Qo)
    assert np.array_equal(host(K).astype(np.uint32), Ko)
    print("[noalloc] subdivision surface, 3 pairs", flush=True)
    (ref, got), _ = both(subdiv_scene(), (16, 256, 0), 3, 5, 1)
    assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])
    assert ref[1].sum() > 0


def test_noalloc_refuses_scratch_beyond_the_array():
    """Per-pair group sums of 5 pairs over a 2048^2 texture (5 x 4.2 M x 8 B)
    exceed the array: DR_E_INVALID, nothing launched."""
    sc = H.quad_scene(np.full((2048, 2048, 3), 0.5, np.float32))
    sc.views = [H.ndc_view(32, 32)]
    ctx = api.Context(sc, DEV)
    theta = dev(sc.flat())
    tg = torch.zeros(3 * 32 * 32, dtype=torch.float32, device=DEV)
    Q, K = ctx.new_accumulators()
    Q.fill_(7)
    K.fill_(3)
    vws = (L.View * 1)(api.make_view(sc.views[0]))
    eps = ctx._eps([1e-3, 1e-2])
    st = ctx.lib.dr_estimate_grad_noalloc(ctx.h, C.c_void_p(theta.data_ptr()), vws, 1, C.c_void_p(tg.data_ptr()),
                                          C.c_uint64(1), C.c_uint32(1), 5, eps, C.c_void_p(Q.data_ptr()),
                                          C.c_void_p(K.data_ptr()))
    assert st == -1
    msg = ctx.lib.dr_last_error(ctx.h).decode()
    assert "maximum" in msg and str(L.NOALLOC_SCRATCH_BYTES) in msg
    assert int((host(Q) != 7).sum()) == 0 and int((host(K) != 3).sum()) == 0
    # one pair fits: the same call then runs and equals dr_estimate_grad
    out = []
    for fn in ("dr_estimate_grad", "dr_estimate_grad_noalloc"):
        Q, K = ctx.new_accumulators()
        st = getattr(ctx.lib, fn)(ctx.h, C.c_void_p(theta.data_ptr()), vws, 1, C.c_void_p(tg.data_ptr()),
                                  C.c_uint64(1), C.c_uint32(1), 1, eps, C.c_void_p(Q.data_ptr()),
                                  C.c_void_p(K.data_ptr()))
        assert st == 0, ctx.lib.dr_last_error(ctx.h)
        out.append((host(Q), host(K)))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert out[0][1].sum() > 0
