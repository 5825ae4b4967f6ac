"""The persistent coarse-step launch's work-distribution protocol, run on host
threads (lbm_persist_model runs the same persist_walk the kernel runs) over the
phase lists the library records for real grids (lbm_plan_phases): the uniform
64x32x32 grid and the three-level 256x128x128 grid of the batching tests.

With the counters zero at the start, every chunk of every phase runs exactly
once, none before the previous phase is complete, and the counters are zero
again at the end, also when the launch has more work-groups than there are
threads to run them at once (work-groups that start late find the work done).

The failure modes: counters that hold stale values at the start (a clear that
is not ordered before the first launch) make every work-group skip the work and
wait; the launch is abandoned after one wait limit and still leaves the counters
zero.  A chunk that never finishes in time makes the others give up within the
wait limit.  A stale `left` count makes the last-to-leave reset fire early, so
chunks run twice: the counters must be cleared on the launch's own stream."""
import time

import numpy as np
import pytest

import oracle as O

GROUPS = 768  # 3 resident work-groups on each of 256 compute units

CASES = {
    "uniform_64x32x32": dict(box=(64, 32, 32), com=(16.0, 16.0, 16.0), L=1, B=16, refine=None),
    "three_level_256x128x128": dict(box=(256, 128, 128), com=(96.0, 64.0, 64.0), L=3, B=8,
                                    refine={"band": [0, 2, 0], "wake": [0, 0, 0]}),
}


@pytest.fixture(scope="module")
def lt():
    import paper_2603_27954_amd as lt
    lt.lib()
    return lt


def _phases(lt, name, steps=4, groups=GROUPS):
    c = CASES[name]
    b = O.build_tree(O.cfg1_tree_params(), 0.0, list(c["com"]))
    nx, ny, nz = c["box"]
    ph = lt.plan_phases(b, groups, coarse_steps=steps, refine=c["refine"], nx=nx, ny=ny, nz=nz, u_in=0.05,
                        re_h=100.0, block_edge=c["B"], levels=c["L"])
    return [[p["chunks"] for p in ph if p["step"] == s] for s in range(steps)], ph


def test_phase_lists_follow_the_coarse_first_schedule(lt):
    """Three levels: per coarse step the collide phases run level 0, 1, 2, 2,
    1, 2, 2 (sub-cycling 1:2:4), each finest sub-step followed by its links and
    force sums, and each level pair ends with its restriction."""
    _, ph = _phases(lt, "three_level_256x128x128", steps=1)
    kinds = [p["kind"] for p in ph]
    assert kinds.count(0) == 7 and kinds.count(1) == 4 and kinds.count(6) == 3
    assert kinds.count(5) == 6 and kinds.count(4) == 3
    _, ph1 = _phases(lt, "uniform_64x32x32", steps=1)
    assert [p["kind"] for p in ph1] == [0, 1, 2, 3]
    assert ph1[0]["items"] == 64 * 32 * 32 // 256


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("threads", [8, 64])
def test_clean_launches_run_every_chunk_once_in_phase_order(lt, name, threads):
    lists, _ = _phases(lt, name)
    ctr = None
    for chunks in lists:  # consecutive launches reuse the counters, as graph replays do
        ctr = np.zeros(2 * len(chunks) + 1, np.uint32) if ctr is None or len(ctr) != 2 * len(chunks) + 1 else ctr
        r, ctr, ab = lt.persist_model(chunks, GROUPS, threads, ctr=ctr, wait_s=5.0)
        assert r["chunks_run"] == sum(chunks)
        assert r["chunks_missed"] == 0 and r["chunks_repeated"] == 0
        assert r["order_violations"] == 0
        assert r["waits_given_up"] == 0 and not r["abandoned"] and ab == 0
        assert r["counters_zero"] and not ctr.any()


def test_more_chunks_than_work_groups_and_fewer_work_groups_than_threads(lt):
    lists, _ = _phases(lt, "three_level_256x128x128", steps=1, groups=5)
    chunks = lists[0]
    assert max(chunks) > 5
    for groups, threads in ((5, 8), (5, 2), (1, 1)):
        r, ctr, ab = lt.persist_model(chunks, groups, threads, wait_s=5.0)
        assert r["chunks_run"] == sum(chunks) and r["chunks_repeated"] == 0 and r["order_violations"] == 0
        assert not r["abandoned"] and r["counters_zero"]


def test_stale_counters_abandon_the_launch_within_the_wait_limit(lt):
    """A claim counter that already reads past the phase's chunk count (a clear
    not yet done when the launch starts) sends every work-group to the next
    wait with the chunks unclaimed: all of them give up after one wait limit,
    nothing runs, and the launch still leaves its counters zero."""
    lists, _ = _phases(lt, "uniform_64x32x32", steps=1)
    chunks = lists[0]
    ctr = np.zeros(2 * len(chunks) + 1, np.uint32)
    ctr[0] = 0xDEADBEEF
    wait_s = 0.2
    t0 = time.time()
    r, ctr, ab = lt.persist_model(chunks, GROUPS, 8, ctr=ctr, wait_s=wait_s)
    assert r["abandoned"] and ab == 1
    assert r["chunks_run"] == 0 and r["waits_given_up"] == GROUPS
    assert wait_s <= r["seconds"] < wait_s + 1.0 and time.time() - t0 < wait_s + 2.0
    assert r["counters_zero"]


def test_stale_left_count_makes_chunks_run_twice(lt):
    """A `left` count that starts above zero makes the last-to-leave reset fire
    while work-groups are still claiming: they claim from zero again and run
    chunks a second time, and the count stays off for the next launch."""
    lists, _ = _phases(lt, "uniform_64x32x32", steps=1)
    chunks = lists[0]
    ctr = np.zeros(2 * len(chunks) + 1, np.uint32)
    ctr[-1] = 100
    r, ctr, _ = lt.persist_model(chunks, GROUPS, 1, ctr=ctr, wait_s=5.0)
    assert r["chunks_repeated"] > 0 or not r["counters_zero"]


def test_a_chunk_that_never_finishes_makes_every_wait_give_up(lt):
    lists, _ = _phases(lt, "three_level_256x128x128", steps=1)
    chunks = lists[0]
    wait_s = 0.1
    r, ctr, ab = lt.persist_model(chunks, GROUPS, 8, wait_s=wait_s, stuck_phase=1)
    assert r["abandoned"] and r["waits_given_up"] > 0
    # the stuck chunks themselves take 3 wait limits; every other work-group
    # leaves after at most one
    n_stuck = chunks[1]
    assert r["seconds"] < (3 * wait_s) * (n_stuck // 8 + 1) + 1.0
    assert r["counters_zero"] and not ctr.any()
    # later phases never started
    assert r["chunks_run"] <= chunks[0] + chunks[1] + chunks[2]
