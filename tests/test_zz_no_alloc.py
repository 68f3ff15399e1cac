"""The deposit entry point that allocates nothing (qh_deposit_noalloc) against qh_deposit, through
the C ABI (needs an MI355X): two calls in a row on the same context, the second with fewer pieces
and points (the static array keeps the first call's contents, which must not leak into the
second), each equal to qh_deposit bit for bit; on the jittered 4^3 box and on the 32^3 cube; a call
beyond the array's size is refused and changes nothing; the context's own deposits are untouched."""
import numpy as np
import pytest

import qh_inputs as qi

from .gpu_setup import chained_segments, gpu_context, oracle_setup

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("wl, counts", [("jitter4", (3000, 700)), ("beam32", (60000, 5000))])
def test_noalloc_deposit_equals_deposit(wl, counts):
    import paper_2103_06737_amd as qh
    cfg = qi.CONFIGS[wl]
    mesh = qi.make_mesh(cfg)
    cx, op, po = oracle_setup(mesh)
    ctx = gpu_context(mesh, cfg["dt"])
    for k, count in enumerate(counts):
        lists = chained_segments(cx, count, 20 + k)
        g_ref, q_ref = ctx.deposit(*lists)
        g, q = ctx.deposit_noalloc(*lists)
        assert np.array_equal(g, g_ref) and np.array_equal(q, q_ref)
        assert g.any() and q.any()
    # empty lists: zero sums even though the array still holds the last call's
    e = np.zeros(0)
    g0, q0 = ctx.deposit_noalloc(e, np.zeros((0, 4)), np.zeros((0, 4)), e, e, np.zeros((0, 4)), e)
    assert not g0.any() and not q0.any()
    # beyond the array (64 MiB): refused, and the next call is still right
    n_big = (64 << 20) // 40 + 1
    big_t = np.zeros(n_big, np.int32)
    big_l = np.zeros((n_big, 4), np.int32)
    big_l[:, 0] = 1 << 20
    with pytest.raises(qh.QhError) as ei:
        ctx.deposit_noalloc(big_t, big_l, big_l, np.ones(n_big, np.int32), np.zeros(0), np.zeros((0, 4)), np.zeros(0))
    assert ei.value.code == qh.QH_EINVAL
    lists = chained_segments(cx, 100, 99)
    g_ref, q_ref = ctx.deposit(*lists)
    g, q = ctx.deposit_noalloc(*lists)
    assert np.array_equal(g, g_ref) and np.array_equal(q, q_ref)
