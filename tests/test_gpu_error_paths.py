"""Error paths of the C ABI on the GPU, forced from the host.

pw_inject_fault(ctx, "alloc" | "launch" | "copy") makes the context fail that class of
HIP call before it is issued, so no kernel ever sees a bad argument.  After each injected failure the
call returns PW_ERR_HIP, and the context keeps its bound state: its results and its
marginal draws afterwards are bitwise those from before.
"""
import numpy as np
import pytest

import synth
from gpu_util import log, make_ctx

pytestmark = pytest.mark.gpu

pw = pytest.importorskip("paper_2601_00761_amd")

ERR_NO_STATE, ERR_HIP = 4, 6
XS = np.array([0, 3, 77, 1000], dtype=np.uint64)


def _snapshot(ctx):
    r = ctx.eval_x(XS, 1e-7)
    d = ctx.sample_x(pw.PW_SAMPLER_MARGINAL_NZ, 11, 0, 256)
    return r.view(np.uint8).copy(), d.copy()


def _same(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("kind", ["launch", "copy"])
def test_injected_failure_in_eval_keeps_the_context(kind):
    ctx = make_ctx(synth.haar_state(12, 1400), pw.PW_C128)
    before = _snapshot(ctx)
    log("eval_x with an injected %s failure" % kind)
    pw.pw_inject_fault(ctx.h, kind)
    with pytest.raises(pw.PWError) as e:
        ctx.eval_x(XS, 1e-7)
    pw.pw_inject_fault(ctx.h, None)
    assert e.value.status == ERR_HIP
    after = _snapshot(ctx)
    ctx.close()
    assert _same(before, after)


def test_injected_failure_in_eval_states_keeps_the_bound_state():
    # the bound state is the largest, so only the pinned staging is allocated (and
    # fails); the workspace is not touched and the bound state comes back intact
    import torch
    ctx = make_ctx(synth.haar_state(14, 1410), pw.PW_C128)
    before = _snapshot(ctx)
    states = [(torch.tensor(synth.haar_state(n, 1420 + n), device="cuda:0"), n, pw.PW_C128) for n in (10, 12)]
    idx = np.array([0, 1, 1], dtype=np.int32)
    xs = np.array([1, 2, 3], dtype=np.uint64)
    for kind in ("alloc", "launch"):
        log("eval_states with an injected %s failure" % kind)
        pw.pw_inject_fault(ctx.h, kind)
        with pytest.raises(pw.PWError) as e:
            pw.pw_eval_states(ctx.h, states, idx, xs, 1e-7)
        pw.pw_inject_fault(ctx.h, None)
        assert e.value.status == ERR_HIP
        assert _same(before, _snapshot(ctx))
    ok = pw.pw_eval_states(ctx.h, states, idx, xs, 1e-7)
    again = pw.pw_eval_states(ctx.h, states, idx, xs, 1e-7)
    ctx.close()
    assert np.array_equal(ok.view(np.uint8), again.view(np.uint8))


def test_failed_workspace_growth_unbinds_and_a_rebind_recovers():
    # a larger state makes eval_states free the library-owned workspace to grow it;
    # with every allocation failing, the bound state cannot be re-carved either, so the
    # context is left without a state; binding the same tensor again restores it
    import torch
    ctx = make_ctx(synth.haar_state(12, 1430), pw.PW_C128)
    before = _snapshot(ctx)
    big = torch.tensor(synth.haar_state(16, 1431), device="cuda:0")
    log("eval_states growing the workspace with an injected alloc failure")
    pw.pw_inject_fault(ctx.h, "alloc")
    with pytest.raises(pw.PWError) as e:
        pw.pw_eval_states(ctx.h, [(big, 16, pw.PW_C128)], np.array([0], dtype=np.int32),
                          np.array([5], dtype=np.uint64), 1e-7)
    pw.pw_inject_fault(ctx.h, None)
    assert e.value.status == ERR_HIP
    with pytest.raises(pw.PWError) as e2:
        ctx.eval_x(XS, 1e-7)
    assert e2.value.status == ERR_NO_STATE
    ctx.bind(ctx.psi, pw.PW_C128)
    after = _snapshot(ctx)
    ctx.close()
    assert _same(before, after)
