"""ldg_jacvec_noalloc (the allocation-free split product) against ldg_jacvec, through the C ABI.

Two calls in a row on one GPU, the second on a smaller problem, so that the shared static scratch
holds the first call's larger w = K21 x when the second runs; with FP64 blocks and the exact tangent,
and with BF16 blocks.  The two entry points run the same kernels on the same inputs, so the outputs
must agree bit for bit.  A problem beyond the scratch size is rejected with LDG_E_UNSUPPORTED.
"""
import numpy as np
import pytest
import torch

from tests.gpu_cases import case, gpu_of

pytestmark = pytest.mark.gpu


def _pair(name, prec, seed):
    pr = case(name)
    ctx = gpu_of(pr)
    U = torch.as_tensor(pr.U0, device="cuda").contiguous()
    ctx.ldg_jacobian_assemble(U, 1.0, 0.02, prec)
    g = torch.Generator(device="cuda").manual_seed(seed)
    x = torch.randn(U.shape, dtype=torch.float64, device="cuda", generator=g)
    out = []
    for exact in (False, True):
        y_ref = torch.empty_like(x)
        y_na = torch.full_like(x, float("nan"))
        ctx.ldg_jacvec(x, y_ref, exact)
        ctx.ldg_jacvec_noalloc(x, y_na, exact)
        torch.cuda.synchronize()
        out.append((exact, y_ref, y_na))
    return ctx, out


@pytest.mark.parametrize("prec", [0, 2])
def test_noalloc_matches_jacvec_on_two_calls_second_smaller(prec):
    print(f"[gpu] jacvec_noalloc prec={prec}", flush=True)
    big, out_big = _pair("tgv2p3", prec, 1)   # E m D Np = 8 * 5 * 3 * 64
    small, out_small = _pair("ns2d_p2", prec, 2)  # 16 * 4 * 2 * 9, a smaller input
    for exact, y_ref, y_na in out_big + out_small:
        assert torch.isfinite(y_na).all()
        assert torch.equal(y_ref, y_na), (exact, float((y_ref - y_na).abs().max()))
    big.close()
    small.close()


def test_noalloc_rejects_problems_beyond_the_scratch():
    from paper_1204_1533_amd import LDGError
    from paper_1204_1533_amd.ldg import LDG_E_UNSUPPORTED
    # E m D Np = 4096 * 5 * 3 * 64 = 3.9 M (the 16^3 p = 3 mesh) fits; 21^3 p = 3 needs 8.9 M
    from ldg_workloads import configs
    big = configs.taylor_green(21, 3, 400.0)
    ctx = gpu_of(big)
    U = torch.as_tensor(big.U0, device="cuda").contiguous()
    ctx.ldg_jacobian_assemble(U, 1.0, 0.02, 2)
    y = torch.empty_like(U)
    with pytest.raises(LDGError) as ei:
        ctx.ldg_jacvec_noalloc(U, y, False)
    assert ei.value.status == LDG_E_UNSUPPORTED
    ctx.close()
