"""Binomial option pricing (out pattern 1 : steps+1) through the C ABI on the
GPU: bit-exact against the oracle for every scheduler, device set and
residency, several tree depths, the plain launch and the paper's full size
(16,777,216 options) sampled."""
import numpy as np
import pytest
import torch

import paper_1805_02755_amd as ce
from paper_1805_02755_amd import synth
from oracle import oracle as O

from gpu_util import BOTH, DEV, check_trace, run_payload

pytestmark = pytest.mark.gpu
DEVSETS = {"gpu": ce.CE_DEV_GPU, "host": ce.CE_DEV_HOST, "both": BOTH}
SIGMA, RATE, T, X = 0.3, 0.05, 1.0, 100.0


@pytest.fixture(scope="module")
def eng():
    e = ce.Engine()
    yield e
    e.close()


def setup(n_groups, steps, seed):
    """The engine gets the library's tree table; the reference is priced on
    the oracle's own table, so the two sides share no input but the spots."""
    spots = synth.binomial_spots(n_groups, seed=seed)
    f, pu, pd = ce.ce_binomial_table(steps, SIGMA, RATE, T)
    fo, puo, pdo = O.binomial_table(steps, SIGMA, RATE, T)
    ref = O.binomial(spots, X, steps, fo, puo, pdo)
    return spots, f, ce.ce_binomial_params(n_groups, steps, X, pu, pd), ref


def same(a, b):
    return np.array_equal(np.ascontiguousarray(a).view(np.uint32), np.ascontiguousarray(b).view(np.uint32))


@pytest.mark.parametrize("mode", ["dev", "host", "both"])
def test_binomial_bitexact_every_schedule(eng, mode):
    spots, f, prm, ref = setup(600, 254, 11)
    for devs in ("gpu", "host", "both"):
        for sched in ("dynamic", "hguided", "static", "static8"):
            out, st, tr = run_payload(eng, ce.CE_KERNEL_BINOMIAL, prm, [255 * 600], [255], [spots, f], (600, 4),
                                      np.float32, DEVSETS[devs], sched, mode=mode)
            assert same(out, ref), (mode, devs, sched)
            check_trace(tr, 600, st.n_devices)


@pytest.mark.parametrize("steps", [1, 2, 3, 63, 64, 65, 127, 128, 129, 191, 192, 193, 200, 254, 255])
def test_binomial_tree_depths(eng, steps):
    spots, f, prm, ref = setup(97, steps, steps)
    out, st, tr = run_payload(eng, ce.CE_KERNEL_BINOMIAL, prm, [(steps + 1) * 97], [steps + 1], [spots, f], (97, 4),
                              np.float32, BOTH, "hguided")
    assert same(out, ref), steps


def test_binomial_plain_launch():
    spots, f, prm, ref = setup(333, 254, 5)
    ins = [torch.from_numpy(spots).to(DEV), torch.from_numpy(f).to(DEV)]
    out = torch.empty((333, 4), device=DEV)
    ce.ce_bare_run(ce.CE_KERNEL_BINOMIAL, prm, ins, out)
    assert same(out.cpu().numpy(), ref)


def test_binomial_paper_size_sampled(eng):
    """16,777,216 options (4,194,304 work-groups of 255), co-executed."""
    n_groups, steps = 4194304, 254
    spots = synth.binomial_spots(n_groups)
    f, pu, pd = ce.ce_binomial_table(steps, SIGMA, RATE, T)
    prm = ce.ce_binomial_params(n_groups, steps, X, pu, pd)
    out, st, tr = run_payload(eng, ce.CE_KERNEL_BINOMIAL, prm, [255 * n_groups], [255], [spots, f], (n_groups, 4),
                              np.float32, BOTH, "dynamic")
    check_trace(tr, n_groups, 2)
    rng = np.random.default_rng(21)
    fo, puo, pdo = O.binomial_table(steps, SIGMA, RATE, T)
    for g in list(rng.choice(n_groups, 40, replace=False)) + [0, n_groups - 1]:
        for c in range(4):
            assert out[g, c].view(np.uint32) == O.binomial_price(float(spots[g, c]), X, steps, fo, puo, pdo).view(
                np.uint32), (g, c)
