"""GPU tests of a sub-domain made of several rectangles, through the C-ABI.

Sec. 3.2 builds the moving bodies' operator on a sub-domain of the finest grid; the sub-domain
may be the union of several rectangles, each moving body taking its P rows on the first
rectangle that holds all of its points (stationary bodies keep the exact operator).  Two
torsional plates far apart, each with a rectangle of its own, stepped against the oracle with
the same rectangles; a plate outside every rectangle is refused; a batch instance with two plates
matches the oracle.
"""
import math

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


def two_plates(n=64, levels=2):
    """Two hinged plates on a 4 x 4 finest level, one upstream left, one down right, with the
    boxes of the sectors they can sweep as two rectangles; a cylinder as a stationary body."""
    h = 4.0 / n
    flow = W.Flow(n=n, levels=levels, h=h, dt=0.2 * h, re=200.0, u_inf=(1.0, 0.0))
    bodies, boxes = [], []
    for hinge, length, th0, inertia in (((-1.4, 0.6), 0.7, math.radians(-20.0), 5.0),
                                       ((0.5, -0.9), 0.6, math.radians(15.0), 3.0)):
        npts = int(round(length / (2.0 * h))) + 1
        bodies.append(W.Torsional(n=npts, hinge=hinge, length=length, theta0=th0,
                                  inertia=inertia, stiffness=1.0, damping=0.1))
        boxes.append(W.plate_box(hinge, length, th0))
    bodies.append(W.cylinder((0.4, 0.9), 0.5, h, spacing=2.0))
    rng = np.random.default_rng(11)
    w0 = [rng.normal(0.0, 1e-3, size=(n - 1, n - 1))] + [None] * (levels - 1)
    return W.Problem("two_rects", flow, bodies, boxes, w0, 3)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_two_plates_in_two_rectangles_match_oracle(torch_cuda, gpu_lib, prec):
    import torch
    from paper_2103_06415_amd import binding
    p = two_plates()
    print(f"two plates, two rectangles {p.subdomain}, n=64 levels 2 {prec}", flush=True)
    iters = 3
    s = binding.Solver(p, precision=binding.IB_FP64 if prec == "fp64" else binding.IB_FP32_FLOW,
                       stream=torch.cuda.Stream(), fixed_iters=iters)
    s.prepare()
    s.step(3)
    s.sync()
    o = Oracle(p, fixed_iters=iters)
    for _ in range(3):
        o.step()
    assert o.sd_body_box == [0, 1, None]
    ev = rel(s.vorticity(0), o.vorticity(0))
    ef = rel(np.concatenate([s.stresses(b) for b in range(3)]), o.f)
    et = max(abs(s.deflection(b)[0] - o.bodies[b][1].theta) for b in (0, 1))
    forces = [s.force(b) for b in range(3)]
    of = o.forces()
    efo = max(float(np.max(np.abs(forces[b] - np.array(of[b])))) /
              max(1e-12, float(np.max(np.abs(of[b])))) for b in range(3))
    st = s.stats()
    print(f"  vorticity {ev:.2e} stresses {ef:.2e} theta {et:.2e} forces {efo:.2e} "
          f"no-slip {st['noslip_resid']:.3e} vs {o.noslip_residual():.3e}", flush=True)
    s.close()
    if prec == "fp64":
        assert ev < 1e-12 and ef < 1e-9 and et < 1e-10 and efo < 1e-9
        assert abs(st["noslip_resid"] - o.noslip_residual()) < 1e-7 * o.noslip_residual()
    else:
        assert ev < 1e-5 and ef < 1e-3 and et < 1e-5 and efo < 1e-3


def test_each_plate_needs_a_rectangle_that_holds_it(torch_cuda, gpu_lib):
    """With only the first plate's rectangle the second plate is outside the sub-domain."""
    from paper_2103_06415_amd import binding
    p = two_plates()
    p.subdomain = [p.subdomain[0]]
    s = binding.Solver(p, precision=binding.IB_FP64)
    with pytest.raises(binding.IbError) as e:
        s.prepare()
    assert e.value.code == binding.IB_ERR_OUT_OF_SUBDOMAIN
    s.close()


def test_batch_instance_with_two_plates_matches_oracle(torch_cuda, gpu_lib):
    """An instance of the batch workload that holds two plates (two rectangles)."""
    import torch
    from paper_2103_06415_amd import binding
    probs = [q for q in W.batch_problems(count=64, sizes=(128,))
             if q.subdomain and len(q.subdomain) >= 2]
    assert probs, "the batch workload draws instances with several plates"
    p = probs[0]
    print(f"{p.name}: n={p.flow.n} levels {p.flow.levels}, {len(p.bodies)} bodies, "
          f"{len(p.subdomain)} rectangles", flush=True)
    s = binding.Solver(p, precision=binding.IB_FP64, stream=torch.cuda.Stream(), fixed_iters=3)
    s.prepare()
    s.step(2)
    s.sync()
    o = Oracle(p, fixed_iters=3)
    for _ in range(2):
        o.step()
    f = np.concatenate([s.stresses(b) for b in range(len(p.bodies))])
    ev, ef = rel(s.vorticity(0), o.vorticity(0)), rel(f, o.f)
    print(f"  vorticity {ev:.2e} stresses {ef:.2e}", flush=True)
    s.close()
    assert ev < 1e-12 and ef < 1e-9
