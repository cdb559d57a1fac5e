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
