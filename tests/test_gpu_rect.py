"""GPU tests of rectangular levels (nx cells along x, ny along y), through the C-ABI.

Sec. 5.3 runs on levels of 4000 x 2000 cells; the solve of Sec. 3.2.1 then takes one sine
transform per axis (rows along x, columns along y) and the nested levels' rings and
coarsification follow their own axes.  Flows without bodies on 2:1 and 1:2 levels with 1-3
levels, stepped against the oracle (FP64 against the long-double oracle at 1e-12 on s and
vorticity, FP32 at 1e-5); bodies and batches are refused on rectangular levels.
"""
import numpy as np
import pytest

import workloads as W
from oracle.step import Oracle

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rect_flow(nx, ny, levels, seed=7):
    h = 4.0 / nx
    flow = W.Flow(n=nx, ny=ny, levels=levels, h=h, dt=0.2 * h, re=250.0, u_inf=(1.0, 0.3))
    rng = np.random.default_rng(seed)
    x = -0.5 * nx * h + h * np.arange(1, nx)
    y = -0.5 * ny * h + h * np.arange(1, ny)
    yy, xx = np.meshgrid(y, x, indexing="ij")
    w = (4.0 * np.exp(-((xx + 0.3) ** 2 + (yy - 0.1) ** 2) / 0.1)
         - 3.0 * np.exp(-((xx - 0.5) ** 2 + (yy + 0.2) ** 2) / 0.05)
         + 0.05 * rng.normal(size=xx.shape))
    return W.Problem("rect", flow, [], vorticity0=[w] + [None] * (levels - 1))


CASES = [(64, 32, 3), (32, 64, 3), (160, 80, 3), (80, 160, 2), (128, 64, 1), (256, 128, 3),
         (40, 20, 2)]
# the long transforms of the paper-scale levels (4000 x 2000) on thin levels the oracle can step:
# rows of 4000 or 2000 (one row per workgroup, ring edges read from memory), columns of 4000 or
# 2000 (one or two columns per workgroup); 4000 in single precision only
BIG = [(4000, 32, 2, "fp32"), (32, 4000, 2, "fp32"), (2000, 64, 2, "fp64"), (2000, 64, 2, "fp32"),
       (64, 2000, 2, "fp64"), (64, 2000, 2, "fp32")]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nx,ny,levels", CASES)
def test_rectangular_flow_matches_oracle(torch_cuda, gpu_lib, nx, ny, levels, prec):
    _check_rect(nx, ny, levels, prec)


def _check_rect(nx, ny, levels, prec):
    import torch
    from paper_2103_06415_amd import binding
    print(f"rectangular flow {nx} x {ny}, {levels} levels, {prec}", flush=True)
    p = rect_flow(nx, ny, levels)
    steps = 4
    s = binding.Solver(p, precision=binding.IB_FP64 if prec == "fp64" else binding.IB_FP32_FLOW,
                       stream=torch.cuda.Stream())
    s.prepare()
    s.step(steps)
    s.sync()
    o = Oracle(p, dtype=np.longdouble if prec == "fp64" else np.float64)
    for _ in range(steps):
        o.step()
    ew = [rel(s.vorticity(g), o.vorticity(g).astype(np.float64)) for g in range(levels)]
    es = [rel(s.streamfunction(g), o.s[g].astype(np.float64)) for g in range(levels)]
    print(f"  vorticity {['%.1e' % e for e in ew]} streamfunction {['%.1e' % e for e in es]}",
          flush=True)
    s.close()
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert max(ew) < tol and max(es) < tol, (ew, es)


def test_rectangular_levels_refuse_bodies_and_batches(torch_cuda, gpu_lib):
    import ctypes
    from paper_2103_06415_amd import binding
    p = rect_flow(64, 32, 1)
    p.bodies = [W.cylinder((0.0, 0.0), 0.5, 4.0 / 64)]
    s = binding.Solver(p, precision=binding.IB_FP64)
    with pytest.raises(binding.IbError) as e:
        s.prepare()
    assert e.value.code == binding.IB_ERR_ARG
    assert "square" in s.last_error()
    s.close()
    q = binding.Solver(rect_flow(64, 32, 1), precision=binding.IB_FP64)
    q.prepare()
    h = ctypes.c_void_p()
    members = (ctypes.c_void_p * 1)(q.handle)
    assert q.lib.ib_batch_create(members, 1, None, ctypes.byref(h)) == binding.IB_ERR_ARG
    assert q.lib.ib_set_flow_variants(q.handle, 1, 0, 0) == binding.IB_ERR_ARG
    q.close()


@pytest.mark.parametrize("nx,ny,levels,prec", BIG)
def test_long_transforms_match_oracle(torch_cuda, gpu_lib, nx, ny, levels, prec):
    _check_rect(nx, ny, levels, prec)
