"""The persistent kernel's grid does not change results: the same outputs,
bit for bit against the oracle, with one workgroup (every tile run in turn
by one workgroup), a few, and more workgroups than the GPU holds at once
(the dispenser's waits must not depend on every workgroup being resident),
for every scheduler over the GPU alone and the GPU with the host."""
import numpy as np
import pytest
import torch

import paper_1805_02755_amd as ce
from paper_1805_02755_amd import synth
from oracle import oracle as O

from gpu_util import BOTH, check_trace, diff_report, escape_params, run_payload

pytestmark = pytest.mark.gpu

GRIDS = [1, 3, 64, 1000, 4096]


@pytest.fixture(scope="module")
def eng():
    e = ce.Engine()
    yield e
    e.close()


@pytest.fixture
def grid(eng, request):
    eng.gpu_workgroups(request.param)
    yield request.param
    eng.gpu_workgroups(0)


@pytest.fixture(scope="module")
def escape_ref():
    p = synth.escape_region(700, 300, -2.0, 0.6, -1.2, 1.2, 400)
    return p, O.escape(p.w, p.h, *[float(v) for v in p.as_f32()], p.max_iter)


@pytest.mark.parametrize("grid", GRIDS, indirect=True)
@pytest.mark.parametrize("sched", ["static8", "dynamic", "hguided"])
@pytest.mark.parametrize("devs", ["gpu", "both"])
def test_escape_any_grid(eng, escape_ref, grid, sched, devs):
    p, ref = escape_ref
    dm = BOTH if devs == "both" else ce.CE_DEV_GPU
    out, st, tr = run_payload(eng, ce.CE_KERNEL_ESCAPE, escape_params(p), [p.w, p.h], None, [], (p.h, p.w),
                              np.uint32, dm, sched)
    assert np.array_equal(out, ref), diff_report(out, ref, tr)
    check_trace(tr, p.h, st.n_devices)
    assert st.gpu_workgroups == grid


@pytest.mark.parametrize("grid", [1, 7, 3000], indirect=True)
@pytest.mark.parametrize("w,h", [(1001, 37), (4099, 23)])
def test_blur_any_grid(eng, grid, w, h):
    img = synth.blur_image(w, h, seed=w + 31 * h)
    wt = ce.ce_gauss5_weights(1.0)
    ref = O.blur5(img, O.gauss5_weights(1.0))
    for sched in ("hguided", "dynamic", "static_rev"):
        out, st, tr = run_payload(eng, ce.CE_KERNEL_BLUR5, ce.ce_blur5_params(w, h), [w, h], None, [img, wt],
                                  (h, w), np.float32, BOTH, sched)
        assert np.array_equal(out.view(np.uint32), ref.view(np.uint32)), (sched, diff_report(out, ref, tr))
        check_trace(tr, h, 2)


@pytest.mark.parametrize("grid", [1, 5, 4096], indirect=True)
def test_nbody_any_grid(eng, grid):
    n = 3000
    pos = synth.nbody_bodies(n, seed=91)
    ref = O.nbody_acc(pos, 1e-6, True)
    for sched in ("dynamic", "hguided", "static"):
        for dm in (ce.CE_DEV_GPU, BOTH):
            out, st, tr = run_payload(eng, ce.CE_KERNEL_NBODY_ACC, ce.ce_nbody_params(n, 1e-6, 1), [n], [256],
                                      [pos], (n, 4), np.float32, dm, sched)
            assert np.array_equal(out.view(np.uint32), ref.view(np.uint32)), (sched, dm)
            check_trace(tr, (n + 255) // 256, st.n_devices)


def _busiest_cu_tiles(tiles, g, cus):
    return -(-tiles // g) * -(-g // cus)


@pytest.mark.parametrize("w,h", [(1024, 1024), (4096, 1024), (2048, 3000), (1000, 77)])
def test_default_grid_balances_the_cus(eng, w, h):
    """Without an override the grid spreads the tiles of the whole space so
    that the busiest compute unit runs no more tiles than it must: with g
    workgroups it runs ceil(T / g) rounds of ceil(g / C) workgroups, and the
    least possible is ceil(T / C) (g = C achieves it); every workgroup gets
    the same number of tiles, give or take one. Checked on escape-time grids
    of 2048, 8192, 12,000 and 154 one-row tiles; the output stays exact."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    eng.gpu_workgroups(0)
    p = synth.escape_region(w, h, -2.0, 1.0, -1.5, 1.5, 64)
    out, st, tr = run_payload(eng, ce.CE_KERNEL_ESCAPE, escape_params(p), [w, h], None, [], (h, w), np.uint32,
                              ce.CE_DEV_GPU, "static")
    ref = O.escape(w, h, *[float(v) for v in p.as_f32()], p.max_iter)
    assert np.array_equal(out, ref), diff_report(out, ref, tr)
    g = st.gpu_workgroups
    tiles = h * -(-w // 512)  # one-row tiles of 512 columns
    assert 0 < g <= tiles
    assert _busiest_cu_tiles(tiles, g, cus) == -(-tiles // cus), (g, tiles, cus)


def test_refuses_huge_grid(eng):
    with pytest.raises(ce.CoexecError):
        eng.gpu_workgroups((1 << 20) + 1)
    eng.clear_errors()
    eng.gpu_workgroups(0)


def test_direct_kernel_one_workgroup_per_tile_over_many_rounds(eng):
    """Equal-cost tiles spanning four or more rounds of resident workgroups,
    the GPU's whole share claimed before the launch: the direct kernel runs
    one workgroup per tile (5120 blur tiles of 32 x 1024 pixels against
    5 x 256 resident workgroups), dealt by the hardware; twice in a row, and
    the whole output bit-exact against the oracle."""
    w, h = 4096, 40960
    img = synth.blur_image(w, h)
    wt = ce.ce_gauss5_weights(1.0)
    ref = O.blur5(img, O.gauss5_weights(1.0))
    for _ in range(2):
        out, st, tr = run_payload(eng, ce.CE_KERNEL_BLUR5, ce.ce_blur5_params(w, h), [w, h], None, [img, wt], (h, w),
                                  np.float32, ce.CE_DEV_GPU, "static")
        assert st.gpu_workgroups == (h // 32) * (w // 1024)
        assert np.array_equal(out.view(np.uint32), ref.view(np.uint32)), diff_report(out, ref, tr)
        check_trace(tr, h, 1)


def test_uneven_tiles_one_workgroup_each_over_many_rounds(eng):
    """Escape-time tiles (uneven cost) over more than four rounds of resident
    workgroups, the GPU alone: the direct kernel runs one workgroup per tile,
    the tiles swizzled over the XCDs (10,005 tiles: the last group of eight
    is partial and keeps its order); twice, the whole image bit-exact."""
    w, h = 2560, 2001
    eng.gpu_workgroups(0)
    p = synth.escape_region(w, h, -2.0, 1.0, -1.5, 1.5, 64)
    ref = O.escape(w, h, *[float(v) for v in p.as_f32()], p.max_iter)
    for _ in range(2):
        out, st, tr = run_payload(eng, ce.CE_KERNEL_ESCAPE, escape_params(p), [w, h], None, [], (h, w), np.uint32,
                                  ce.CE_DEV_GPU, "static")
        assert st.gpu_workgroups == h * -(-w // 512)
        assert np.array_equal(out, ref), diff_report(out, ref, tr)
        check_trace(tr, h, 1)
