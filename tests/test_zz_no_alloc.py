"""The allocation-free prox trial (fb_lisa_step_noalloc) against the plan-based entry point
(fb_lisa_step), through the C ABI: two calls in a row, the second on a smaller volume, for
each storage type.  The kernels are the same, so outputs and reductions agree bit for bit."""
import ctypes
import math

import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fbl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2605_12085_amd as fbl
    return fbl


@pytest.mark.parametrize("st", ["f32", "bf16", "f16"])
def test_noalloc_step_matches_plan_step(fbl, st):
    import torch
    from paper_2605_12085_amd import _lib
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[st]
    code = {"f32": _lib.FBL_F32, "bf16": _lib.FBL_BF16, "f16": _lib.FBL_F16}[st]
    # a volume of 1,064,895 voxels (2048 blocks and several grid-stride passes here, 1040
    # one-pass blocks in the plan's trial; a ragged tail after the four-voxel groups), then
    # a small one
    big = syn.Geometry(127, 129, 65, 0.5, 0.5, 0.5, 192, 192, 0.5, 0.5, 500.0, 1000.0, 4)
    small = syn.Geometry(13, 11, 7, 1.0, 1.0, 1.0, 20, 16, 1.5, 1.5, 300.0, 600.0, 4)
    rng = np.random.default_rng(70)
    settings = [(2.5e-3, 0.7, 0.0, 0.03), (1e-3, 0.0, 0.0, math.inf)]
    for call, (geom, (alpha, mu, lo, hi)) in enumerate(zip((big, small), settings)):
        print("no-alloc step: storage %s, call %d, %d voxels" % (st, call, geom.d), flush=True)
        x = torch.from_numpy(rng.uniform(0, 0.03, geom.vol_shape).astype(np.float32)).to(tdt).cuda()
        g = torch.from_numpy((rng.standard_normal(geom.vol_shape) * 3.0).astype(np.float32)).cuda()
        xb_n = torch.full_like(x, float("nan"))
        red_n = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
        rc = _lib.lib.fb_lisa_step_noalloc(x.numel(), code, x.data_ptr(), g.data_ptr(), alpha, mu, lo, hi,
                                           xb_n.data_ptr(), red_n.data_ptr(), _lib._stream(None))
        assert rc == 0, _lib.lib.fbl_last_error().decode()
        with fbl.Plan(geom, vol_dtype=st, max_batch=1) as plan:
            xb_p, red_p = fbl.fb_lisa_step(plan, x, g, alpha, mu, lo, hi)
            torch.cuda.synchronize()
        # the trial points agree bit for bit; the FP64 sums are added over different block
        # partitions (the plan's trial runs one pass of four voxels per thread, this one a
        # grid-stride loop over at most 2048 blocks), so they agree to FP64 rounding
        assert torch.equal(xb_n, xb_p)
        rn, rp = red_n.cpu().numpy(), red_p.cpu().numpy()
        assert np.all(np.abs(rn - rp) <= 1e-12 * np.abs(rp)), (rn, rp)
    # size and argument checks launch nothing
    x = torch.zeros(8, dtype=tdt, device="cuda")
    g = torch.zeros(8, dtype=torch.float32, device="cuda")
    xb = torch.zeros(8, dtype=tdt, device="cuda")
    red = torch.zeros(3, dtype=torch.float64, device="cuda")
    assert _lib.lib.fb_lisa_step_noalloc(1 << 31, code, x.data_ptr(), g.data_ptr(), 1e-3, 0.0, 0.0, math.inf,
                                         xb.data_ptr(), red.data_ptr(), None) == _lib.FBL_E_RANGE
    assert "2^31" in _lib.lib.fbl_last_error().decode()
    assert _lib.lib.fb_lisa_step_noalloc(0, code, x.data_ptr(), g.data_ptr(), 1e-3, 0.0, 0.0, math.inf,
                                         xb.data_ptr(), red.data_ptr(), None) == _lib.FBL_E_RANGE
    assert _lib.lib.fb_lisa_step_noalloc(8, 7, x.data_ptr(), g.data_ptr(), 1e-3, 0.0, 0.0, math.inf,
                                         xb.data_ptr(), red.data_ptr(), None) == _lib.FBL_E_DTYPE
    assert _lib.lib.fb_lisa_step_noalloc(8, code, x.data_ptr(), g.data_ptr(), -1.0, 0.0, 0.0, math.inf,
                                         xb.data_ptr(), red.data_ptr(), None) == _lib.FBL_E_INVALID
