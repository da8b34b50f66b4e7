"""lbm_reduce_noalloc, the reduction that allocates nothing, against
lbm_reduce through the C ABI (needs an MI355X: -m gpu).  Both run the same
kernels in the same order, so the sums agree bit for bit; two calls in a row
on contexts of decreasing size (the second sees the first call's leftovers
in the shared work array), at FP64 and FP32, and the refusal of a context
with more blocks than the work array holds."""
import numpy as np
import pytest

from paper_1711_03254_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1711_03254_amd.lbm as m
    m.load_library()
    return m


def _ctx(lbm, torch, shape, prec, seed, stream):
    nz, ny, nx = shape
    solid = inputs.random_mask(shape, 0.1, seed)
    solid[:, 0, :] = 1
    r1 = inputs.smooth_random_density(shape, seed + 1, mean=0.6, amp=0.25)
    r2 = 1.0 - r1
    u = 0.03 * (inputs.uniform(seed + 2, 3 * r1.size).reshape((3,) + shape) - 0.5)
    r1[solid == 1] = 0
    r2[solid == 1] = 0
    ctx = lbm.lbm_init(lbm.Params(nx, ny, nz, prec=lbm.PRECISIONS[prec], solid=solid, rho_init=(r1, r2), u_init=u,
                                  tau=(0.7, 1.3), G=-2.5, g=(1e-5, 0.0, 2e-5), rho_s=0.2, stream=stream))
    lbm.lbm_step(ctx, 3)
    return ctx


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_reduce_noalloc_equals_reduce(lbm, prec):
    import torch
    stream = torch.cuda.Stream()
    for k, shape in enumerate([(40, 33, 70), (9, 12, 17)]):   # the second call on a smaller context
        ctx = _ctx(lbm, torch, shape, prec, 100 + 10 * k, stream)
        want = lbm.lbm_reduce(ctx)
        out = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        lbm.lbm_reduce_noalloc(ctx, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, want), (shape, got, want)
        lbm.lbm_free(ctx)


def test_reduce_noalloc_refuses_too_many_blocks(lbm):
    import torch
    # 8 x 32 tiles on 64 x 64 planes: 16 tile columns; one plane per z-chunk
    # over 1100 planes gives 17600 blocks, more than the 16384 the work
    # array holds.  Refused on the host, before any device work.
    shape = (1100, 64, 64)
    nz, ny, nx = shape
    r = np.full(shape, 0.5)
    ctx = lbm.lbm_init(lbm.Params(nx, ny, nz, prec=lbm.LBM_FP32, rho_init=(r, r.copy()), tile=(8, 32), zchunk=1))
    assert lbm.lbm_info(ctx)["blocks"] == 17600
    out = torch.zeros(5, dtype=torch.float64, device="cuda")
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_reduce_noalloc(ctx, out)
    assert e.value.code == lbm.LBM_EINVAL and "16384" in str(e.value)
    lbm.lbm_free(ctx)
