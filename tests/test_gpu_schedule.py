"""Transform schedules (pw_set_schedule) and the schedule autotuner through the C ABI.

Every plan variant that applies to a state (first pass over 12 or 15 index bits, column
tiles of 12 / 13 / 15 bits) is checked against the FP64 oracle on the same input (single
precision within the fp_bounds bound, double precision at 1e-10 relative, nullity counts
exact), and the first-pass tile-sharing groups of 2, 4, 8 and 16 families against group 1 of
the same plan bitwise.  The autotuner's choice is one of the candidates, survives
pw_autotune_save / pw_autotune_load, and reaches a new context.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from fp_bounds import family_bounds_from_sums
from gpu_util import as_input, log, make_ctx

pytestmark = pytest.mark.gpu
pw = pytest.importorskip("paper_2601_00761_amd")


def _plans(n, dtype):
    nh = n - 1
    if dtype == pw.PW_C128:
        return [(12, 12)]
    out = [(12, 12), (12, 13)]
    sb = nh - 15
    if 1 <= sb <= 12:
        if sb <= 8:
            out.append((15, 12))
        if sb <= 9:
            out.append((15, 13))
        if sb >= 9:
            out.append((15, 15))
    return out


def _xs(n, seed):
    w = synth.splitmix64(seed, 0, 15) % np.uint64(1 << n)
    return np.array([0] + [int(v) for v in w], dtype=np.uint64)


@pytest.mark.parametrize("n,dtype", [(17, pw.PW_C64), (20, pw.PW_C64), (23, pw.PW_C64), (26, pw.PW_C64),
                                     (18, pw.PW_C128), (22, pw.PW_C128)])
def test_every_schedule_matches_the_oracle(n, dtype):
    psi = synth.haar_state(n, 8000 + n)
    xs = _xs(n, 8100 + n)
    eps = 1e-7 if dtype == pw.PW_C128 else 1e-4
    ctx = make_ctx(psi, dtype, x_batch=16)
    r = oracle.eval_x_with_bound_sums(as_input(psi, dtype), xs, eps=eps, max_alpha=4)
    for fb, ct in _plans(n, dtype):
        base = None
        for g in (1, 2, 4, 8, 16):
            pw.pw_set_schedule(ctx.h, fb, ct, g, 16)
            got = pw.pw_get_schedule(ctx.h)
            log("schedule n=%d dtype=%d first=%d column=%d group=%d -> %s" % (n, dtype, fb, ct, g, got))
            assert got[:2] == (fb, ct) and got[3] == 16
            assert got[2] == g or (g > 1 and got[2] < g)
            res = ctx.eval_x(xs, eps)
            if base is None:
                base = res
                for i in range(len(xs)):
                    if dtype == pw.PW_C128:
                        assert abs(res["m"][i, 0] / r["m"][i, 0] - 1) < 1e-10
                        assert abs(res["p"][i] / r["p"][i] - 1) < 1e-10
                    else:
                        b = family_bounds_from_sums(r, i, n)
                        assert abs(res["m"][i, 0] - r["m"][i, 0]) <= b["m2"]
                        assert abs(res["p"][i] - r["p"][i]) <= b["p"]
                        assert abs(res["ent"][i] - r["ent"][i]) <= b["ent"]
                    assert int(res["nu"][i]) == int(r["nu"][i])
            else:
                assert np.array_equal(res.view(np.uint8), base.view(np.uint8)), (fb, ct, g)
    ctx.close()


def test_set_schedule_rejects_what_does_not_apply():
    ctx = make_ctx(synth.haar_state(18, 8200), pw.PW_C128)
    for args, status in (((15, 0, 0, 0), 8), ((12, 13, 0, 0), 8), ((11, 0, 0, 0), 1), ((0, 0, 3, 0), 1),
                         ((0, 0, 256, 0), 1), ((0, 0, 0, -1), 1)):
        with pytest.raises(pw.PWError) as e:
            pw.pw_set_schedule(ctx.h, *args)
        assert e.value.status == status, args
    ctx.close()


def test_autotune_schedule_persists(tmp_path):
    # (n = 21 complex64: no later test compares a context's results at this size bitwise
    # with another path, and the tuned schedule stays in the process)
    n = 21
    psi = synth.haar_state(n, 8300).astype(np.complex64)
    ctx = make_ctx(psi, pw.PW_C64, x_batch=16)
    best, table = pw.pw_autotune(ctx.h)
    sched = pw.pw_get_schedule(ctx.h)
    log("autotune n=%d best batch %d schedule %s table %s" % (n, best, sched, table))
    assert sched[3] == best and best in table
    assert (sched[0], sched[1]) in _plans(n, pw.PW_C64)
    path = os.path.join(str(tmp_path), "tune.txt")
    pw.pw_autotune_save(path)
    with open(path) as f:
        lines = [ln for ln in f if not ln.startswith("#")]
    assert any(ln.split()[1:3] == [str(n), "1"] for ln in lines)
    assert pw.pw_autotune_load(path) >= 1
    ctx.close()
    # a new context on a state of the same size takes the tuned schedule
    ctx2 = make_ctx(psi, pw.PW_C64, x_batch=16)
    assert pw.pw_get_schedule(ctx2.h) == sched
    ctx2.close()
