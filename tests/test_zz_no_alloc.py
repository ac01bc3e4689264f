"""The allocation-free operator solve (ib_op_solve_noalloc) against ib_op_solve and the oracle.

Both entry points run the same kernels on the same tables, so their outputs agree bit for bit;
both are held to the oracle's [L (I + alpha L)]^{-1} (Sec. 3.2.1, eqs. (30)-(31)) at the
operator bars (1e-13 in double, 2e-6 in single precision).  Calls come in a row on one GPU,
the largest tables first (n = 1280 in double), then a smaller single-precision case, then an
in-place call, so each call reuses the fixed device array the previous one wrote.
"""
import numpy as np
import pytest

from oracle import dst

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


CASES = [(1280, "fp64", 3, False), (96, "fp32", 7, False), (64, "fp64", 0, True)]


def test_noalloc_solve_equals_the_allocating_one(torch_cuda, gpu_lib):
    torch = torch_cuda
    from paper_2103_06415_amd import binding
    stream = torch.cuda.current_stream().cuda_stream
    for n, prec, pad, in_place in CASES:
        print(f"noalloc op solve n={n} {prec} pitch n-1+{pad} in_place={in_place}", flush=True)
        rng = np.random.default_rng(n)
        x = rng.normal(size=(n - 1, n - 1))
        alpha = 0.05
        pitch = n - 1 + pad
        dtype = torch.float64 if prec == "fp64" else torch.float32
        code = binding.IB_FP64 if prec == "fp64" else binding.IB_FP32_FLOW
        src = torch.zeros((n - 1, pitch), dtype=dtype, device="cuda")
        src[:, : n - 1] = torch.from_numpy(x).to(dtype)
        ref_out = torch.zeros_like(src)
        binding.op_solve(n, code, alpha, src.data_ptr(), ref_out.data_ptr(), pitch, stream)
        if in_place:
            got = src.clone()
            binding.op_solve_noalloc(n, code, alpha, got.data_ptr(), got.data_ptr(), pitch, stream)
        else:
            got = torch.full_like(src, float("nan"))
            binding.op_solve_noalloc(n, code, alpha, src.data_ptr(), got.data_ptr(), pitch, stream)
        torch.cuda.synchronize()
        a = got[:, : n - 1].double().cpu().numpy()
        b = ref_out[:, : n - 1].double().cpu().numpy()
        xo = x if prec == "fp64" else x.astype(np.float32).astype(np.float64)
        o = dst.solve_cac(xo, alpha)
        e = rel(a, o)
        print(f"  bitwise equal to ib_op_solve: {np.array_equal(a, b)}; against the oracle {e:.2e}",
              flush=True)
        assert np.array_equal(a, b)
        assert e < (1e-13 if prec == "fp64" else 2e-6), e


def test_noalloc_solve_rejects_bad_arguments(torch_cuda, gpu_lib):
    from paper_2103_06415_amd import binding
    lib = binding.load()
    assert lib.ib_op_solve_noalloc(100, binding.IB_FP64, 0.1, None, None, 99, None) == -1
    assert lib.ib_op_solve_noalloc(64, 7, 0.1, None, None, 63, None) == -1
