"""Batched form (one persistent, graph-captured launch over many uneven
escape-time jobs): parity with the oracle, invariance over tile shapes and
package sizes, graph replays, autotuner, the per-job baseline and errors."""
import numpy as np
import pytest
import torch

import paper_1805_02755_amd as ce
from paper_1805_02755_amd import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _params(p):
    return ce.ce_escape_params(p.w, p.h, *p.as_f32(), p.max_iter)


def _ref(p):
    return O.escape(p.w, p.h, *[float(v) for v in p.as_f32()], p.max_iter)


@pytest.fixture(scope="module")
def small_jobs():
    jobs = synth.batch_jobs(24, seed=77, side_lo=5, side_hi=300, iter_lo=20, iter_hi=600)
    return jobs, [_ref(p) for p in jobs]


def _make(jobs):
    b = ce.Batch()
    outs = []
    for p in jobs:
        o = torch.full((p.h, p.w), -1, dtype=torch.int32, device=DEV)
        outs.append(o)
        b.add_escape(_params(p), o)
    torch.cuda.synchronize()
    return b, outs


def _check(outs, refs):
    for i, (o, r) in enumerate(zip(outs, refs)):
        assert np.array_equal(o.cpu().numpy().view(np.uint32), r), i


def test_batch_matches_oracle_every_config(small_jobs):
    jobs, refs = small_jobs
    b, outs = _make(jobs)
    for rows in (1, 2, 4, 8, 16):
        for pkg in (1, 7, 32):
            for o in outs:
                o.fill_(-1)
            torch.cuda.synchronize()
            b.set_config(rows, pkg)
            b.run()
            _check(outs, refs)
            st = b.stats()
            assert st.tile_rows == rows and st.tile_cols * rows == 256 and st.package_tiles == pkg
            assert st.items == sum(p.w * p.h for p in jobs) and st.jobs == len(jobs)
    b.close()


def test_graph_replays_with_eager_work_between(small_jobs):
    jobs, refs = small_jobs
    b, outs = _make(jobs)
    b.set_config(4, 4)
    for rep in range(5):
        for o in outs:
            o.zero_()  # eager work on torch's stream between replays
        torch.cuda.synchronize()
        b.run()
        _check(outs, refs)
    assert b.stats().launches == 5
    b.close()


def test_separate_launch_baseline_matches(small_jobs):
    jobs, refs = small_jobs
    b, outs = _make(jobs)
    b.run_separate()
    _check(outs, refs)
    b.close()


def test_autotuner_picks_a_valid_config(small_jobs):
    jobs, refs = small_jobs
    b, outs = _make(jobs)
    rows, cols, pkg = b.tune(reps=1)
    assert rows in (1, 2, 4, 8, 16) and rows * cols == 256 and pkg >= 1
    for o in outs:
        o.fill_(-1)
    torch.cuda.synchronize()
    b.run()
    _check(outs, refs)
    b.close()


def test_full_size_batch_sampled():
    jobs = synth.batch_jobs()
    assert len(jobs) == 256
    b, outs = _make(jobs)
    b.set_config(16, 4)
    b.run()
    rng = np.random.default_rng(5)
    for p, o in zip(jobs, outs):
        a = o.cpu().numpy().view(np.uint32)
        for r, c in [(0, 0), (p.h - 1, p.w - 1)] + [(int(rng.integers(p.h)), int(rng.integers(p.w))) for _ in range(3)]:
            want = O.escape_pixel(r, c, *[float(v) for v in p.as_f32()], p.max_iter)
            assert a[r, c] == want, (p, r, c)
        assert a.min() >= 1 and a.max() <= p.max_iter
    b.close()


def test_batch_errors():
    b = ce.Batch()
    with pytest.raises(ce.CoexecError) as ei:
        b.run()
    assert ei.value.status == ce.CE_E_STATE
    o = torch.zeros(4, dtype=torch.int32, device=DEV)
    with pytest.raises(ce.CoexecError) as ei:
        b.add_escape(ce.ce_escape_params(0, 4, 0, 0, 1, 1, 5), o)
    assert ei.value.status == ce.CE_E_INVALID
    with pytest.raises(ce.CoexecError) as ei:
        b.set_config(3, 4)
    assert ei.value.status == ce.CE_E_INVALID
    b.close()
