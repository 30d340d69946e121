"""Serving form (continuous batching on one persistent serving kernel):
outputs of jobs admitted while others run are bit-identical to the oracle's
and to the same job run alone; HBM-budget and in-flight admission limits
hold; jobs submitted together run at the same time on the device; sessions
restart, roll over when full and end when idle; invalid and oversized jobs
are refused."""
import time

import numpy as np
import pytest
import torch

import paper_1805_02755_amd as ce
from paper_1805_02755_amd import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
MiB = 1 << 20
SESSION_S = 60.0  # the serving kernel leaves by itself after this long without a new job


def _esc(p):
    return ce.ce_escape_params(p.w, p.h, *p.as_f32(), p.max_iter)


def _esc_ref(p):
    return O.escape(p.w, p.h, *[float(v) for v in p.as_f32()], p.max_iter)


class Job:
    """One job of a test mix: how to submit it and what it must produce."""

    def __init__(self, kind, params, ins, ref, shape, dtype):
        self.kind, self.params, self.ins, self.ref, self.shape, self.dtype = kind, params, ins, ref, shape, dtype

    def upload(self):
        """Device copies of the inputs, read in place by the serving kernel."""
        self.dev = [torch.from_numpy(a).to(DEV) for a in self.ins]
        torch.cuda.synchronize()

    def submit(self, srv, resident=False):
        return srv.submit(self.kind, self.params, *(self.dev if resident else self.ins))

    def check(self, srv, ticket):
        srv.wait(ticket, 60.0)
        out = np.empty(self.shape, self.dtype)
        srv.copy_output(ticket, out)
        assert np.array_equal(out.view(np.uint32), self.ref.view(np.uint32)), (self.kind, self.shape)
        return out


def escape_job(w, h, it, box=(-2.0, 0.6, -1.2, 1.2)):
    p = synth.escape_region(w, h, *box, it)
    return Job(ce.CE_KERNEL_ESCAPE, _esc(p), [], _esc_ref(p), (h, w), np.uint32)


def blur_job(w, h, wt=None):
    """Gaussian weights by default (the library's for the job, the oracle's
    for the reference; a CPU test pins the two bitwise), else ``wt``."""
    img = synth.blur_image(w, h, seed=w * 31 + h)
    if wt is None:
        wt, wt_ref = ce.ce_gauss5_weights(1.0), O.gauss5_weights(1.0)
    else:
        wt_ref = wt
    return Job(ce.CE_KERNEL_BLUR5, ce.ce_blur5_params(w, h), [img, wt], O.blur5(img, wt_ref), (h, w), np.float32)


def nbody_job(n):
    pos = synth.nbody_bodies(n, seed=n + 3)
    return Job(ce.CE_KERNEL_NBODY_ACC, ce.ce_nbody_params(n, 1e-6, 1), [pos], O.nbody_acc(pos, 1e-6, True),
               (n, 4), np.float32)


@pytest.fixture(scope="module")
def mix():
    rng = np.random.default_rng(9)
    jobs = [escape_job(w, h, it) for (w, h, it) in [(64, 16, 200), (333, 77, 700), (1, 1, 50), (1024, 40, 300),
                                                    (65, 17, 1000), (700, 300, 256)]]
    jobs += [blur_job(w, h) for (w, h) in [(203, 77), (1001, 37), (4099, 23), (5, 5)]]
    jobs.append(blur_job(517, 61, rng.random(25).astype(np.float32)))
    jobs += [nbody_job(n) for n in (7, 1000, 4097)]
    order = rng.permutation(len(jobs))
    return [jobs[i] for i in order]


def test_mixed_jobs_match_oracle(mix):
    with ce.Server(256 * MiB, keep_outputs=True, session_timeout_s=SESSION_S) as srv:
        tickets = [j.submit(srv) for j in mix]
        for j, t in zip(mix, tickets):
            j.check(srv, t)
            srv.release(t)
        srv.drain(60.0)
        r = srv.stats()
        assert r.submitted == r.completed == len(mix)
        assert r.items == sum(int(np.prod(j.shape[:2])) if j.kind != ce.CE_KERNEL_NBODY_ACC else j.shape[0]
                              for j in mix)
        assert 0 < r.peak_hbm <= 256 * MiB
        assert r.p50_s <= r.p99_s <= r.max_s and r.items_per_s > 0


def test_resident_device_inputs(mix):
    with ce.Server(64 * MiB, keep_outputs=True, session_timeout_s=SESSION_S) as srv:
        for j in mix:
            j.upload()  # before the first submit starts the session
        tickets = [j.submit(srv, resident=True) for j in mix]
        for j, t in zip(mix, tickets):
            j.check(srv, t)
        srv.drain(60.0)


def test_alone_and_in_a_mix_give_the_same_bytes(mix):
    target = next(j for j in mix if j.kind == ce.CE_KERNEL_BLUR5 and j.shape == (37, 1001))
    with ce.Server(64 * MiB, keep_outputs=True, session_timeout_s=SESSION_S) as srv:
        alone = target.check(srv, target.submit(srv))
        srv.drain(60.0)
    with ce.Server(256 * MiB, keep_outputs=True, session_timeout_s=SESSION_S) as srv:
        tickets = [j.submit(srv) for j in mix]
        outs = {id(j): j.check(srv, t) for j, t in zip(mix, tickets)}
        srv.drain(60.0)
    assert np.array_equal(alone.view(np.uint32), outs[id(target)].view(np.uint32))


def test_budget_limits_admission():
    jobs = [escape_job(256, 256, 64 + 37 * i) for i in range(24)]  # 256 KiB output each
    budget = 2 * 256 * 1024 + 1024
    with ce.Server(budget, keep_outputs=True, session_timeout_s=SESSION_S) as srv:
        tickets = [j.submit(srv) for j in jobs]
        for j, t in zip(jobs, tickets):
            j.check(srv, t)
            srv.release(t)  # frees the job's memory: the next job can be admitted
        srv.drain(60.0)
        r = srv.stats()
        assert r.completed == len(jobs)
        assert r.peak_hbm <= budget
        assert 1 <= r.max_inflight_seen <= 2


def test_in_flight_limit_and_freeing_on_completion():
    jobs = [escape_job(100 + 13 * i, 50 + 7 * i, 300) for i in range(12)]
    with ce.Server(32 * MiB, max_inflight=1, keep_outputs=False, session_timeout_s=SESSION_S) as srv:
        tickets = [j.submit(srv) for j in jobs]
        for t in tickets:
            srv.wait(t, 60.0)
        with pytest.raises(ce.CoexecError) as ei:
            srv.output(tickets[0])
        assert ei.value.status == ce.CE_E_STATE  # freed when it finished
        srv.drain(60.0)
        r = srv.stats()
        assert r.completed == len(jobs) and r.max_inflight_seen == 1


def test_sessions_restart():
    a, b = escape_job(129, 33, 500), nbody_job(300)
    with ce.Server(16 * MiB, keep_outputs=True, session_timeout_s=SESSION_S) as srv:
        a.check(srv, a.submit(srv))
        srv.drain(60.0)
        b.check(srv, b.submit(srv))
        a.check(srv, a.submit(srv))
        srv.drain(60.0)
        assert srv.stats().completed == 3


def test_refused_jobs():
    with ce.Server(1 * MiB, keep_outputs=True, session_timeout_s=SESSION_S) as srv:
        with pytest.raises(ce.CoexecError) as ei:
            srv.submit(ce.CE_KERNEL_ESCAPE, ce.ce_escape_params(1024, 1024, -2, -1, 0.01, 0.01, 10))
        assert ei.value.status == ce.CE_E_BUDGET  # 4 MiB of output
        with pytest.raises(ce.CoexecError) as ei:
            srv.submit(ce.CE_KERNEL_ESCAPE, ce.ce_escape_params(0, 4, -2, -1, 0.01, 0.01, 10))
        assert ei.value.status == ce.CE_E_INVALID
        with pytest.raises(ce.CoexecError) as ei:
            srv.submit(ce.CE_KERNEL_BLUR5, ce.ce_blur5_params(8, 8))  # no image
        assert ei.value.status == ce.CE_E_INVALID
        with pytest.raises(ce.CoexecError) as ei:
            srv.submit(ce.CE_KERNEL_NBODY_ACC, ce.ce_nbody_params(8, 0.0, 1), synth.nbody_bodies(8))
        assert ei.value.status == ce.CE_E_INVALID
        with pytest.raises(ce.CoexecError) as ei:
            srv.wait(12345, 0.1)
        assert ei.value.status == ce.CE_E_INVALID
        srv.drain(10.0)  # no session was started: nothing to do


def test_full_size_jobs_sampled():
    """The largest job of each kind in the serving trace's size ranges."""
    esc = synth.escape_region(4096, 4096, -2.0, 1.0, -1.5, 1.5, 4096)
    img = synth.blur_image(16384, 16384, seed=3)
    wt, wt_ref = ce.ce_gauss5_weights(1.0), O.gauss5_weights(1.0)
    pos = synth.nbody_bodies(131072, seed=5)
    with ce.Server(3 << 30, keep_outputs=True, session_timeout_s=SESSION_S) as srv:
        te = srv.submit(ce.CE_KERNEL_ESCAPE, _esc(esc))
        tb = srv.submit(ce.CE_KERNEL_BLUR5, ce.ce_blur5_params(16384, 16384), img, wt)
        tn = srv.submit(ce.CE_KERNEL_NBODY_ACC, ce.ce_nbody_params(131072, 1e-6, 1), pos)
        for t in (te, tb, tn):
            srv.wait(t, 60.0)
        oe = srv.copy_output(te, np.empty((4096, 4096), np.uint32))
        ob = srv.copy_output(tb, np.empty((16384, 16384), np.float32))
        on = srv.copy_output(tn, np.empty((131072, 4), np.float32))
        srv.drain(60.0)
    rng = np.random.default_rng(11)
    for r, c in [(0, 0), (4095, 4095), (2048, 1365)] + [tuple(rng.integers(4096, size=2)) for _ in range(12)]:
        assert oe[r, c] == O.escape_pixel(int(r), int(c), *[float(v) for v in esc.as_f32()], 4096)
    assert oe.min() >= 1 and oe.max() <= 4096
    for y, x in [(0, 0), (16383, 16383), (0, 16383), (7, 9000)] + [tuple(rng.integers(16384, size=2)) for _ in range(40)]:
        assert ob[y, x].view(np.uint32) == O.blur5_pixel(img, wt_ref, int(y), int(x)).view(np.uint32)
    for i in [0, 131071] + list(rng.integers(131072, size=6)):
        assert np.array_equal(on[i].view(np.uint32), O.nbody_acc_body(pos, 1e-6, int(i), True).view(np.uint32))


def test_concurrent_jobs_overlap_on_the_device():
    """Continuous batching: jobs admitted together share the GPU, so the
    [first tile, last tile] intervals of at least two of them overlap, and
    more than one job was in flight at once."""
    jobs = [escape_job(1024, 512, 3000 + 100 * i) for i in range(4)] + [blur_job(4096, 1024), nbody_job(20000)]
    with ce.Server(512 * MiB, keep_outputs=True, session_timeout_s=SESSION_S) as srv:
        tickets = [j.submit(srv) for j in jobs]
        for j, t in zip(jobs, tickets):
            j.check(srv, t)
        spans = [srv.job_ticks(t) for t in tickets]
        srv.drain(60.0)
        r = srv.stats()
    assert all(0 < a <= b for a, b in spans), spans
    overlaps = sum(1 for i in range(len(spans)) for k in range(i + 1, len(spans))
                   if spans[i][0] < spans[k][1] and spans[k][0] < spans[i][1])
    assert overlaps >= 1, spans
    assert r.max_inflight_seen >= 2


def test_sessions_roll_over_when_full():
    """A session takes max_jobs jobs; the server thread ends it and starts the
    next for the rest, so ten jobs through sessions of four all complete."""
    jobs = [escape_job(200 + 11 * i, 90, 300 + 50 * i) for i in range(10)]
    with ce.Server(64 * MiB, keep_outputs=True, max_jobs=4, session_timeout_s=SESSION_S) as srv:
        tickets = [j.submit(srv) for j in jobs]
        for j, t in zip(jobs, tickets):
            j.check(srv, t)
        srv.drain(60.0)
        assert srv.stats().completed == 10


def test_idle_session_ends_and_the_next_job_starts_another():
    a, b = escape_job(300, 100, 400), blur_job(1001, 37)
    with ce.Server(32 * MiB, keep_outputs=True, session_timeout_s=0.2) as srv:
        a.check(srv, a.submit(srv))
        time.sleep(0.6)  # the kernel has left: no job for 0.2 s
        b.check(srv, b.submit(srv))
        a.check(srv, a.submit(srv))
        srv.drain(30.0)
        assert srv.stats().completed == 3
