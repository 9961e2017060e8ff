"""fpde_apply_noalloc (the apply for callers that cannot allocate) against fpde_apply.

Two calls in a row through the C ABI, the second on a smaller operator (the
static scratch keeps the first call's contents, which the entry point must
clear), in FP64 and in mixed precision, FP64 and FP32 vectors: the output equals
fpde_apply's bit for bit (same kernels, workspace in the static scratch).  The
entry point rejects nrhs != 1, an operator without far blocks, and a workspace
above the 8 MiB scratch.
"""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from fpde_inputs import configs  # noqa: E402


def _plain(op, x):
    import paper_2302_02863_amd as fp
    y = torch.empty_like(x)
    dt = fp._abi.F64 if x.dtype is torch.float64 else fp._abi.F32
    st = fp._abi.lib().fpde_apply(op._h, dt, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), 1,
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    fp._abi.check(st, "fpde_apply")
    return y


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_apply_two_calls(precision):
    import paper_2302_02863_amd as fp
    cases = [configs.square(24, 12, leaf_size=16, leaf_size_rho=32, cheb_p=4),
             configs.square(12, 6, leaf_size=16, leaf_size_rho=32, cheb_p=4)]
    for P in cases:   # larger first, then smaller
        o = dict(P.opts)
        o["precision"] = precision
        op = fp.Operator(P.mesh, P.s, P.kappa, o)
        assert op.stats()["k_far"] > 0
        for dtype in (torch.float64, torch.float32):
            x = torch.tensor(P.x, device="cuda", dtype=dtype)
            y_ref = _plain(op, x)
            y = torch.full_like(x, float("nan"))
            op.apply_noalloc(x, y)
            y2 = torch.full_like(x, float("nan"))
            op.apply_noalloc(x, y2)
            torch.cuda.synchronize()
            print(f"[noalloc] {precision} N={P.mesh.n_dofs} {dtype}: max |diff| "
                  f"{float((y - y_ref).abs().max()):.3e}", flush=True)
            assert torch.equal(y, y_ref) and torch.equal(y2, y_ref)
        op.close()


def test_noalloc_rejections():
    import paper_2302_02863_amd as fp
    P = configs.square(12, 6, leaf_size=16, leaf_size_rho=32, cheb_p=4)
    op = fp.Operator(P.mesh, P.s, P.kappa, P.opts)
    x = torch.zeros((1, op.n_dofs, 2), device="cuda", dtype=torch.float64)
    st = fp._abi.lib().fpde_apply_noalloc(op._h, fp._abi.F64, C.c_void_p(x.data_ptr()),
                                          C.c_void_p(x.data_ptr() + 8), 2, None)
    assert st == fp._abi.FPDE_EINVAL and b"nrhs" in fp._abi.lib().fpde_last_error()
    op.close()
    P = configs.square(4, 2, leaf_size=16, leaf_size_rho=32, cheb_p=3)   # no far blocks
    op = fp.Operator(P.mesh, P.s, P.kappa, P.opts)
    assert op.stats()["k_far"] == 0
    x = torch.zeros((1, op.n_dofs, 1), device="cuda", dtype=torch.float64)
    with pytest.raises(fp._abi.FpdeError, match="one-vector path"):
        op.apply_noalloc(x, torch.empty_like(x))
    op.close()
    # 8 fields of the 128 x 128 square with leaves of 16 need about 14 MiB of workspace
    P = configs.batched(128, n_fields=8, nrhs=1, leaf_size=16, leaf_size_rho=64)
    op = fp.Operator(P.mesh, P.s, P.kappa, P.opts)
    x = torch.zeros((8, op.n_dofs, 1), device="cuda", dtype=torch.float64)
    with pytest.raises(fp._abi.FpdeError, match="bytes of workspace"):
        op.apply_noalloc(x, torch.empty_like(x))
    op.close()
