"""Graph-captured batches with the convergence test on the device.

* slab_batch_run: the factorization of every problem of an uneven batch and
  all refinement passes of its solve as one HIP graph launch; replayed three
  times with eager work and synchronizations in between, the last two after
  new coefficient fields were written into the same buffers, it equals an
  eager factorization and solve of the same fields (and the oracle).
* SLAB_GRAPH batch solves with several refinement passes (all-FP32 form):
  the device-side test stops each problem at the pass the host test stops it.
* A non-positive coefficient written into the buffers of problem 1 between
  replays is reported for problem 1.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gen import inputs as G
from oracle import slab_oracle as O
from paper_2211_07572_amd import slab as S

pytestmark = pytest.mark.gpu

DIMS = [(40, 48, 7, 2), (70, 96, 15, 1), (130, 128, 31, 3), (33, 24, 1, 4), (64, 64, 7, 5),
        (5, 4, 3, 1), (96, 160, 15, 2)]


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _inputs(seed0):
    kaps = [G.kappa_lognormal(n2, n1, seed0 + i) for i, (n2, n1, b, _) in enumerate(DIMS)]
    fs = [G.rhs_uniform(n2, n1, nr, seed0 + 50 + i) for i, (n2, n1, b, nr) in enumerate(DIMS)]
    return kaps, fs


def _eager(kaps, fd, precision):
    bt = S.slab_factor_batch([_dev(k) for k in kaps], [d[:3] for d in DIMS], precision=precision)
    us = [u.cpu().numpy() for u in S.slab_solve_batch(bt, fd)]
    its = [i.iterations for i in bt.last_infos]
    bt.free()
    return us, its


@pytest.mark.parametrize("precision", [S.SLAB_FP64, S.SLAB_MIXED, S.SLAB_FP32_REFINE])
def test_batch_run_graph_replays(precision):
    kaps_a, fs = _inputs(80)
    kaps_b, _ = _inputs(90)
    fd = [_dev(f) for f in fs]
    kbuf = [_dev(k) for k in kaps_a]
    bt = S.slab_factor_batch(kbuf, [d[:3] for d in DIMS], precision=precision, tol=1e-10)
    outs = [torch.empty_like(f) for f in fd]
    for rep, kaps in enumerate((kaps_a, kaps_b, kaps_b)):
        print(f"batch run: precision {precision}, replay {rep}", flush=True)
        for kb, k in zip(kbuf, kaps):
            kb.copy_(_dev(k))                 # new fields into the captured buffers
        for o in outs:
            o.fill_(float(rep + 1))           # eager work between the replays
        torch.cuda.synchronize()
        us = S.slab_batch_run(bt, kbuf, fd, outs=outs)
        torch.cuda.synchronize()
        ref, ref_it = _eager(kaps, fd, precision)
        for i, (n2, n1, b, nr) in enumerate(DIMS):
            u = us[i].cpu().numpy()
            assert np.array_equal(u, ref[i]), (rep, i)
            assert bt.last_infos[i].iterations == ref_it[i], (rep, i)
            rr = O.relres(O.make_problem(kaps[i], n2, n1, b), u, fs[i]).max()
            assert rr <= 1e-10, (rep, i, rr)
    # the batch's handles hold the factors of the last fields
    u1 = S.slab_solve(bt.handle(2), fd[2]).cpu().numpy()
    assert np.array_equal(u1, ref[2])
    bt.free()


def test_graph_solve_stops_each_problem_like_the_host():
    kaps, fs = _inputs(100)
    fd = [_dev(f) for f in fs]
    ref, ref_it = _eager(kaps, fd, S.SLAB_FP32_REFINE)
    assert max(ref_it) > 1   # several passes, so the device-side test matters
    bt = S.slab_factor_batch([_dev(k) for k in kaps], [d[:3] for d in DIMS],
                             precision=S.SLAB_FP32_REFINE, graph=True)
    for rep in range(2):
        us = S.slab_solve_batch(bt, fd)
        for i in range(len(DIMS)):
            assert bt.last_infos[i].iterations == ref_it[i], (rep, i)
            assert np.array_equal(us[i].cpu().numpy(), ref[i]), (rep, i)
    bt.free()


def test_batch_run_reports_invalid_field():
    kaps, fs = _inputs(110)
    fd = [_dev(f) for f in fs]
    kbuf = [_dev(k) for k in kaps]
    bt = S.slab_factor_batch(kbuf, [d[:3] for d in DIMS], precision=S.SLAB_MIXED)
    S.slab_batch_run(bt, kbuf, fd)
    kbuf[1][3, 4] = -1.0
    with pytest.raises(S.SlabError) as ei:
        S.slab_batch_run(bt, kbuf, fd)
    assert ei.value.status == S.SLAB_E_INVALID
    assert "problem 1" in str(ei.value)
    bt.free()
