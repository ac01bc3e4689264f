"""GPU parity at the sizes the throughput measurement runs: 1024^2 x 4 levels and
512^2 x 3 levels, three steps of the flow (predictor with nested-level rings, Sec. 2.3
eq. (16), Sec. 3.2.1 transforms, Sec. 5 far field) against the FP64 oracle.

Single precision runs every measured transform configuration (the kernel instances the
throughput measurement picks from at these sizes), the configuration it picked in the
latest measurement (rows 7, columns 5, inverse rows 7) and the choice ib_prepare measures
itself; the bar is the FP32 form's 1e-5 on the vorticity.  Double precision is compared
with the oracle run in extended precision (long double): the double-precision oracle
re-differences its streamfunction for the circulation it hands between levels and so
carries errors of up to 1e-10 of its own at these sizes.  The bar is 1e-12 for the
vorticity and for the streamfunction (relative L2 over each level; s with its ring).

Bodies at a size where the measured configurations apply (n >= 256): a short torsional
plate and a short flag at 256^2 x 2 in sub-domain mode with a fixed FSI iteration count,
so that the oracle can build B' column by column in seconds.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle.step import Oracle

pytestmark = pytest.mark.gpu

STEPS = 3
EPS64 = 2.0 ** -52


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def fp64_vorticity_tol(n, steps):
    return max(1e-12, 40.0 * EPS64 * 0.5 * (n / math.pi) ** 2 * math.sqrt(steps))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _flow_problem(n, levels, seed=7):
    """A Gaussian vortex plus N(0, 0.05^2) noise on the finest level, free stream (1, 0.3)."""
    rng = np.random.default_rng(seed)
    flow = W.Flow(n=n, levels=levels, h=3.2 / n, dt=0.2 * 3.2 / n, re=150.0, cx=0.1, cy=-0.05,
                  u_inf=(1.0, 0.3))
    x = flow.cx - 0.5 * n * flow.h + flow.h * np.arange(1, n)
    y = flow.cy - 0.5 * n * flow.h + flow.h * np.arange(1, n)
    yy, xx = np.meshgrid(y, x, indexing="ij")
    w = 4.0 * np.exp(-((xx + 0.2) ** 2 + (yy - 0.1) ** 2) / 0.08) + 0.05 * rng.normal(size=xx.shape)
    return W.Problem("flow", flow, [], vorticity0=[w] + [None] * (levels - 1))


_ORACLE = {}


def _oracle(n, levels, dtype=np.float64):
    key = (n, levels, np.dtype(dtype).name)
    if key not in _ORACLE:
        print(f"oracle flow n={n} levels={levels} {STEPS} steps {np.dtype(dtype).name}", flush=True)
        o = Oracle(_flow_problem(n, levels), dtype=dtype)
        for _ in range(STEPS):
            o.step()
        _ORACLE[key] = ([o.vorticity(g).astype(np.float64) for g in range(levels)],
                        [o.s[g].astype(np.float64) for g in range(levels)])
    return _ORACLE[key]


SIZES = [(512, 3), (1024, 4)]
CONFIGS = ["measured", (7, 5, 7)] + [(v, v, v) for v in range(8)]
# the register-resident column solve (configuration 8) exists at n = 1024 only
CASES = [(n, lv, c) for n, lv in SIZES for c in CONFIGS] + [(1024, 4, (7, 8, 7)), (1024, 4, (0, 8, 0))]


@pytest.mark.parametrize("n,levels,config", CASES,
                         ids=lambda c: c if isinstance(c, str) else ("-".join(map(str, c)) if isinstance(c, tuple) else str(c)))
def test_fp32_transform_configurations_at_bench_sizes(torch_cuda, gpu_lib, n, levels, config):
    from paper_2103_06415_amd import binding
    w_ref, s_ref = _oracle(n, levels)
    print(f"fp32 flow n={n} levels={levels} config={config}", flush=True)
    s = binding.Solver(_flow_problem(n, levels), precision=binding.IB_FP32_FLOW)
    if config != "measured":
        s.set_flow_variants(*config)
    s.prepare()
    t = s.flow_tuning()
    if config != "measured":
        assert (t["rhs_variant"], t["col_variant"], t["idst_variant"]) == config
    s.step(STEPS)
    s.sync()
    errs = [rel(s.vorticity(g), w_ref[g]) for g in range(levels)]
    serrs = [rel(s.streamfunction(g), s_ref[g]) for g in range(levels)]
    print(f"  chosen {t['rhs_variant']},{t['col_variant']},{t['idst_variant']}: vorticity rel L2 "
          f"{max(errs):.2e}, streamfunction {max(serrs):.2e}", flush=True)
    s.close()
    assert max(errs) < 1e-5, errs


@pytest.mark.parametrize("n,levels", SIZES)
def test_fp64_at_bench_sizes(torch_cuda, gpu_lib, n, levels):
    from paper_2103_06415_amd import binding
    w_ref, s_ref = _oracle(n, levels, np.longdouble)
    w64, s64 = _oracle(n, levels)
    print(f"fp64 flow n={n} levels={levels}", flush=True)
    s = binding.Solver(_flow_problem(n, levels), precision=binding.IB_FP64)
    s.prepare()
    s.step(STEPS)
    s.sync()
    serrs = [rel(s.streamfunction(g), s_ref[g]) for g in range(levels)]
    werrs = [rel(s.vorticity(g), w_ref[g]) for g in range(levels)]
    o_s = [rel(s64[g], s_ref[g]) for g in range(levels)]
    o_w = [rel(w64[g], w_ref[g]) for g in range(levels)]
    print(f"  against the extended-precision oracle: streamfunction rel L2 {serrs}; vorticity "
          f"{werrs}; the double oracle itself: streamfunction {o_s}, vorticity {o_w}", flush=True)
    s.close()
    assert max(serrs) < 1e-12, serrs
    assert max(werrs) < 1e-12, werrs


def _short_body_problem(which, n=256, levels=2):
    """A 5.12-wide finest level at n = 256 (h = 0.02, dt = 0.2 h), Re 200, a body of length
    0.28 with points 2h apart and a tight sub-domain around it."""
    width = 5.12
    h = width / n
    flow = W.Flow(n=n, levels=levels, h=h, dt=0.2 * h, re=200.0, cx=0.5, cy=0.0)
    length = 0.28
    if which == "plate":
        npts = int(round(length / (2.0 * h))) + 1
        th0 = -math.radians(20.0)
        body = W.Torsional(n=npts, hinge=(0.0, 0.0), length=length, theta0=th0, inertia=0.5,
                           stiffness=1.0, damping=0.1, theta=0.02, phi=0.1)
        sd = W.plate_box((0.0, 0.0), length, th0, spread=math.radians(30.0))
    else:
        body = W.flag_body((0.0, 0.0), length, h, mass=0.2, ei=1e-3, a=0.02)
        sd = (-0.02, length + 0.02, -0.12, 0.12)
    rng = np.random.default_rng(21)
    w0 = [rng.normal(0.0, 1e-3, size=(n - 1, n - 1))] + [None] * (levels - 1)
    return W.Problem(which, flow, [body], sd, w0, STEPS)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("which", ["plate", "flag"])
def test_bodies_at_a_tuned_size(torch_cuda, gpu_lib, which, prec):
    from paper_2103_06415_amd import binding
    iters = 3
    p = _short_body_problem(which)
    print(f"{which} n=256 levels=2 {prec} fixed iterations {iters}", flush=True)
    s = binding.Solver(p, precision=binding.IB_FP64 if prec == "fp64" else binding.IB_FP32_FLOW,
                       fixed_iters=iters)
    s.prepare()
    t = s.flow_tuning()
    s.step(STEPS)
    s.sync()
    ora = Oracle(p, fixed_iters=iters)
    for _ in range(STEPS):
        ora.step()
    st = s.stats()
    errs = [rel(s.vorticity(g), ora.vorticity(g)) for g in range(2)]
    ef = rel(s.stresses(0), ora.f)
    d = s.deflection(0)
    b = ora.bodies[0][1]
    ed = abs(d[0] - b.theta) if which == "plate" else float(np.max(np.abs(d - b.chi)))
    print(f"  tuning {t['rhs_variant']},{t['col_variant']},{t['idst_variant']}; nnz "
          f"{st['subdomain_nnz']} vs {np.count_nonzero(ora.b_filtered)}; vorticity {errs}; "
          f"stresses {ef:.2e}; deflection {ed:.2e}", flush=True)
    s.close()
    assert st["subdomain_nnz"] == int(np.count_nonzero(ora.b_filtered))
    assert max(errs) < (fp64_vorticity_tol(256, STEPS) if prec == "fp64" else 1e-5)
    assert ef < (1e-9 if prec == "fp64" else 1e-3)
    assert ed < (1e-10 if prec == "fp64" else 1e-5)
