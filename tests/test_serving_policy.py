"""Host logic of the serving scheduler: which admitted jobs may start their next
chunk under each policy (no device work)."""
import types

import pytest

from paper_1901_06503_amd.serving import Scheduler, _remaining_work


class _C:
    def __init__(self, n):
        self.n = n

    def numel(self):
        return self.n ** 3


def _active(job_id, arrival, n, done=0, n_iter=50, powered=True, nt=100):
    job = types.SimpleNamespace(job_id=job_id, arrival=arrival, c=_C(n), n_iter=n_iter, n_power=20)
    a = types.SimpleNamespace(job=job, done_iters=done, powered=powered, plan=types.SimpleNamespace(nt=nt))
    return a


def _ids(chosen):
    return [a.job.job_id for a in chosen]


def test_fill_runs_in_arrival_order_up_to_the_threshold():
    s = Scheduler(hbm_budget=1 << 30, policy="fill", fill_voxels=192 ** 3)
    act = [_active(3, 0.3, 64), _active(1, 0.1, 128), _active(2, 0.2, 128), _active(4, 0.4, 64)]
    # 128^3 + 128^3 = 4.2M <= 7.1M; + 64^3 (0.26M) still fits
    assert _ids(s._choose(act)) == [1, 2, 3, 4]
    big = [_active(5, 0.0, 256), _active(6, 0.1, 64)]
    assert _ids(s._choose(big)) == [5]                    # the oldest always runs, even alone
    mid = [_active(7, 0.0, 192), _active(8, 0.1, 64), _active(9, 0.2, 128)]
    assert _ids(s._choose(mid)) == [7]                    # 192^3 + 64^3 > 192^3: nothing joins
    tie = [_active(11, 0.0, 64), _active(10, 0.0, 64)]
    assert _ids(s._choose(tie)) == [10, 11]               # equal arrivals: by job id


def test_fill_stops_at_the_first_job_that_does_not_fit():
    s = Scheduler(hbm_budget=1 << 30, policy="fill", fill_voxels=160 ** 3)
    act = [_active(1, 0.0, 128), _active(2, 0.1, 128), _active(3, 0.2, 64)]
    assert _ids(s._choose(act)) == [1]                    # no overtaking past job 2


def test_shortest_keeps_the_oldest_and_adds_the_least_remaining_work():
    s = Scheduler(hbm_budget=1 << 30, policy="shortest", concurrency=2, aging=0.0, low_concurrency=2)
    act = [_active(1, 0.0, 256), _active(2, 0.1, 128, done=40), _active(3, 0.2, 64)]
    rem = {a.job.job_id: _remaining_work(a) for a in act}
    assert rem[3] < rem[2] < rem[1]
    assert _ids(s._choose(act)) == [1, 3]


def test_shortest_ages_waiting_jobs():
    # priority = remaining work in seconds (at 4e11 point updates per second) minus the
    # time waited, i.e. arrival + remaining work: a job is overtaken only by jobs that
    # arrive less than its remaining work minus theirs later.  A 256^3 job with 50
    # iterations left (2 * 171 * 256^3 * 50 = 2.9e11: 0.72 s) that arrived at 1.0 goes
    # before a 64^3 job (0.007 s) arriving at 1.8, after one arriving at 1.5
    s = Scheduler(hbm_budget=1 << 30, policy="shortest", concurrency=2, aging=1.0, low_concurrency=2)
    s._now = 2.0
    late = [_active(1, 0.0, 128, done=10), _active(2, 1.0, 256, nt=171), _active(3, 1.8, 64)]
    assert _ids(s._choose(late)) == [1, 2]
    early = [_active(1, 0.0, 128, done=10), _active(2, 1.0, 256, nt=171), _active(3, 1.5, 64)]
    assert _ids(s._choose(early)) == [1, 3]
    s.aging = 0.0                                          # no aging: least remaining work
    assert _ids(s._choose(late)) == [1, 3]


def test_remaining_work_counts_the_power_iteration():
    a = _active(1, 0.0, 64, powered=False)
    b = _active(1, 0.0, 64, powered=True)
    assert _remaining_work(a) == pytest.approx(_remaining_work(b) * 70 / 50)


def test_all_and_unknown_policy():
    s = Scheduler(hbm_budget=1 << 30, policy="all")
    act = [_active(2, 0.1, 256), _active(1, 0.0, 256)]
    assert _ids(s._choose(act)) == [2, 1]
    with pytest.raises(ValueError):
        Scheduler(hbm_budget=1, policy="lifo")


def test_shortest_runs_more_jobs_only_under_a_backlog():
    s = Scheduler(hbm_budget=1 << 30, policy="shortest", concurrency=3, backlog=3, aging=0.0, low_concurrency=2,
                  join_voxels=0)
    act = [_active(1, 0.0, 256), _active(2, 0.1, 64), _active(3, 0.2, 128), _active(4, 0.3, 192)]
    s._waiting = 3                                         # few jobs in the system: two at a time
    assert _ids(s._choose(act)) == [1, 2]
    s._waiting = 6                                         # a queue has formed: three
    assert _ids(s._choose(act)) == [1, 2, 3]


def test_shortest_below_the_backlog_by_default():
    # below the device's capacity the default runs the oldest job, as the serial
    # baseline does, plus only jobs of at most 128^3 points (their small launches leave
    # the device mostly idle; sharing it with larger jobs slows the long ones)
    s = Scheduler(hbm_budget=1 << 30, policy="shortest", aging=0.0)
    assert s.backlog == 5 and s.low_concurrency == 1 and s.concurrency == 3 and s.join_voxels == 128 ** 3
    act = [_active(1, 0.0, 256), _active(2, 0.1, 192), _active(3, 0.2, 256), _active(4, 0.3, 192)]
    s._waiting = 5
    assert _ids(s._choose(act)) == [1]
    s._waiting = 6
    assert _ids(s._choose(act)) == [1, 2, 4]
    mixed = [_active(1, 0.0, 256), _active(2, 0.1, 64), _active(3, 0.2, 128), _active(4, 0.3, 192)]
    s._waiting = 5
    assert _ids(s._choose(mixed)) == [1, 2, 3]


def test_small_jobs_join_the_oldest_below_the_backlog():
    # join_voxels: below the backlog, jobs of at most that many grid points run beside
    # the oldest (up to `concurrency` jobs), in the policy's order; larger ones wait
    s = Scheduler(hbm_budget=1 << 30, policy="shortest", aging=0.0, join_voxels=128 ** 3)
    act = [_active(1, 0.0, 256), _active(2, 0.1, 192), _active(3, 0.2, 128), _active(4, 0.3, 64),
           _active(5, 0.4, 64)]
    s._waiting = 5
    assert _ids(s._choose(act)) == [1, 4, 5]              # the two 64^3 jobs: least remaining work
    s._waiting = 6                                         # above the backlog: unchanged rule
    assert _ids(s._choose(act)) == [1, 4, 5]
    s.join_voxels = 0
    s._waiting = 5
    assert _ids(s._choose(act)) == [1]
    s.join_voxels = 128 ** 3
    big_only = [_active(1, 0.0, 256), _active(2, 0.1, 192)]
    assert _ids(s._choose(big_only)) == [1]


def test_chunks_hold_at_least_min_chunk_s_of_device_work():
    # 2 solves x n_t x points per iteration at 4e11 point updates per second: a 64^3
    # job (n_t 42, 55 us per iteration) takes all its 50 iterations in one chunk, a
    # 128^3 job (n_t 85, 0.89 ms) 23, a 256^3 job (n_t 170, 14 ms) the minimum of 5
    s = Scheduler(hbm_budget=1 << 30, iters_per_turn=5, min_chunk_s=0.02)
    assert s._chunk(_active(1, 0.0, 64, nt=42)) == 50
    assert s._chunk(_active(2, 0.0, 128, nt=85)) == 23
    assert s._chunk(_active(3, 0.0, 256, nt=170)) == 5
    assert s._chunk(_active(4, 0.0, 128, nt=85, done=40)) == 10      # what is left
    s.min_chunk_s = 0.0
    assert s._chunk(_active(5, 0.0, 64, nt=42)) == 5
