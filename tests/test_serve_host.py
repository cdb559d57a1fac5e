"""Host logic of the serving loop: admission control and arrivals (no GPU)."""
import numpy as np
import pytest

from paper_2012_12686_amd.serve import Admission, poisson_arrivals


def test_admission_respects_budget_jobs_and_positions():
    adm = Admission(budget_bytes=1000, max_jobs=3, max_positions=100)
    assert adm.try_admit(400, 60)
    assert not adm.try_admit(700, 10)          # over the HBM budget
    assert not adm.try_admit(100, 50)          # over the positions per tick
    assert adm.try_admit(500, 40)
    assert not adm.try_admit(150, 0)           # 400 + 500 + 150 > 1000
    adm.release(400, 60)
    assert adm.used == 500 and adm.jobs == 1 and adm.positions == 40
    assert adm.try_admit(100, 10) and adm.try_admit(100, 10)
    assert not adm.try_admit(1, 1)             # three jobs already
    assert adm.fits_ever(1000) and not adm.fits_ever(1001)


def test_a_lone_job_may_exceed_the_positions_cap():
    adm = Admission(budget_bytes=10, max_jobs=4, max_positions=8)
    assert adm.try_admit(5, 50)                # the first job always fits the slots
    assert not adm.try_admit(1, 1)
    adm.release(5, 50)
    with pytest.raises(AssertionError):
        adm.release(5, 50)


def test_poisson_arrivals_statistics():
    t = poisson_arrivals(4.0, 20000, seed=3)
    gaps = np.diff(t)
    assert t[0] == 0.0 and np.all(gaps >= 0)
    assert abs(gaps.mean() - 0.25) < 0.01                  # rate 4 / s
    assert abs(gaps.std() - 0.25) < 0.01                   # exponential: std = mean
    assert np.array_equal(t, poisson_arrivals(4.0, 20000, seed=3))


class _Geom:
    def __init__(self, n, n_slices):
        self.n, self.n_slices = n, n_slices


class _Tpl:
    """The fields of a job type that admission and job_work read."""

    def __init__(self, n, n_slices, minibatch, shape, kind="scan"):
        import torch
        self.geom = _Geom(n, n_slices)
        self.a0 = torch.empty(shape, device="meta")
        self.minibatch = minibatch
        self.kind = kind


def _requests():
    from paper_2012_12686_amd.serve import Request
    big = _Tpl(192, 256, 100, (256, 512, 512))
    small = _Tpl(64, 64, 16, (64, 128, 128))
    tilt = _Tpl(128, 128, 25, (128, 256, 256), kind="tilt")
    return [Request(0.0, big, 20), Request(0.1, small, 20), Request(0.2, tilt, 20), Request(0.3, small, 5)]


def test_job_work_orders_job_types_by_their_sweep_and_voxels():
    from paper_2012_12686_amd.serve import job_work
    big, small, tilt, short = _requests()
    w = [job_work(r.template, r.iterations) for r in (big, small, tilt, short)]
    assert w[3] < w[1] < w[2] < w[0]
    assert w[3] == pytest.approx(w[1] * 5 / 20)           # linear in the iterations
    # the sweep term: positions x slices x N^2 log2 N, plus 2 Adam passes per voxel
    assert w[1] == pytest.approx(20 * (16 * 64 * 64 * 64 * 6 + 2 * 64 * 128 * 128))
    # a tilt job also rotates the object and its gradient each iteration
    assert w[2] == pytest.approx(20 * (25 * 128 * 128 * 128 * 7 + 6 * 128 * 256 * 256))


@pytest.mark.parametrize("order", ["fifo", "sjf"])
def test_admission_order(order):
    from paper_2012_12686_amd.serve import Server
    reqs = _requests()
    foot = [600, 100, 300, 100]
    srv = Server(ctx=None, budget_bytes=1000, max_jobs=3, max_positions=10_000, order=order)
    waiting = [0, 1, 2, 3]
    got = []
    while (i := srv._admit_next(waiting, reqs, foot)) is not None:
        got.append(i)
    if order == "fifo":
        # the head is admitted, then the next in arrival order while they fit
        assert got == [0, 1, 2] and waiting == [3]
    else:
        # least work first; the big job no longer fits behind the three others
        assert got == [3, 1, 2] and waiting == [0]
    assert srv.adm.jobs == 3


def test_fifo_head_that_does_not_fit_blocks_the_rest_and_sjf_does_not():
    from paper_2012_12686_amd.serve import Server
    reqs = _requests()
    foot = [900, 100, 300, 100]
    for order, admitted in (("fifo", []), ("sjf", [3, 1, 2])):
        srv = Server(ctx=None, budget_bytes=1000, max_jobs=4, max_positions=10_000, order=order)
        assert srv.adm.try_admit(300, 1)                  # a running job holds 300
        waiting = [0, 1, 2, 3]
        got = []
        while (i := srv._admit_next(waiting, reqs, foot)) is not None:
            got.append(i)
        assert got == admitted


def test_unknown_order_is_refused():
    from paper_2012_12686_amd.serve import Server
    with pytest.raises(ValueError):
        Server(ctx=None, budget_bytes=1000, order="lifo")


def test_slot_limit_rises_with_a_deep_queue():
    from paper_2012_12686_amd.serve import Server
    reqs = _requests() * 2                       # 8 requests, 100 bytes each
    foot = [100] * len(reqs)
    srv = Server(ctx=None, budget_bytes=10_000, max_jobs=2, max_positions=10_000, busy_jobs=4, busy_queue=6)
    waiting = list(range(len(reqs)))
    got = []
    while (i := srv._admit_next(waiting, reqs, foot)) is not None:
        got.append(i)
    # 8 and 7 waiting: the busy limit of 4 applies; 6 waiting: still busy; then
    # 5 waiting falls back to 2 slots, already taken
    assert got == [0, 1, 2] and srv.adm.jobs == 3
    srv.adm.release(100, 1)
    waiting = waiting[:2]                        # a short queue
    assert srv._admit_next(waiting, reqs, foot) is None and srv.adm.max_jobs == 2
    with pytest.raises(ValueError):
        Server(ctx=None, budget_bytes=1000, max_jobs=4, busy_jobs=2)


def test_the_served_form_of_the_bench_is_a_valid_configuration():
    from paper_2012_12686_amd.serve import SERVED, Server
    srv = Server(ctx=None, budget_bytes=10_000, **SERVED)
    assert srv.streams == SERVED["streams"] >= 1
    assert srv.max_jobs <= srv.busy_jobs and srv.busy_queue >= 1
    assert srv.order == "fifo"                 # the long jobs are the tail: no least-work-first
