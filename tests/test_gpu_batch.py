"""Batches (ib_batch_*): many solvers stepped with one launch per kernel for all members.

Every member's results must equal those of the same solver stepped alone, bit for bit: the
batched launches run the same kernels on the same per-member arguments.  The alone runs
are themselves held to the FP64 oracle by the parity tests; one batched member is also
checked against the oracle directly here.
"""
import numpy as np
import pytest

import workloads as W
from oracle.step import Oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _flow_only(n, levels, seed):
    rng = np.random.default_rng(seed)
    flow = W.Flow(n=n, levels=levels, h=3.2 / n, dt=0.2 * 3.2 / n, re=150.0, cx=0.1, cy=-0.05,
                  u_inf=(1.0, 0.3))
    w0 = [rng.normal(0.0, 1e-2, size=(n - 1, n - 1)) for _ in range(levels)]
    return W.Problem("flow", flow, [], None, w0, 0)


def _members():
    """Uneven sizes, level counts and body kinds: stationary circles, torsional plates,
    a deformable flag, a driven (moving) plate, the driven plate with a passive plate on its
    hinge, a body-less flow and config-4 style instances with several bodies."""
    probs = [
        W.cylinder_problem(n=32, steps=0),
        W.plate_problem(n=48, levels=2, steps=0),
        W.flag_problem(n=64, levels=2, steps=0),
        W.driven_plate_problem(n=64, levels=2, steps=0),
        W.two_plate_problem(n=64, levels=2, steps=0, case=1),
        _flow_only(32, 3, 7),
        W.cylinder_problem(n=32, seed=9, steps=0),
    ]
    probs += W.batch_problems(count=4, seed=11, steps=0, sizes=(32, 48, 64))
    return probs


def _prec(prec):
    from paper_2103_06415_amd import binding
    return binding.IB_FP64 if prec == "fp64" else binding.IB_FP32_FLOW


def _results(s, p):
    out = {}
    for g in range(p.flow.levels):
        out[f"w{g}"] = s.vorticity(g)
    for b in range(len(p.bodies)):
        out[f"f{b}"] = s.stresses(b)
        out[f"d{b}"] = s.deflection(b)
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batched_members_equal_their_runs_alone(torch_cuda, gpu_lib, prec):
    from paper_2103_06415_amd import binding
    steps = 7
    probs = _members()
    alone = []
    for k, p in enumerate(probs):
        print(f"alone {prec} member {k} {p.name} n={p.flow.n} levels={p.flow.levels}", flush=True)
        s = binding.Solver(p, precision=_prec(prec))
        s.prepare()
        s.step(steps)
        s.sync()
        alone.append(_results(s, p))
        s.close()
    print(f"batch {prec} of {len(probs)} members, {steps} steps", flush=True)
    sols = []
    for p in probs:
        s = binding.Solver(p, precision=_prec(prec))
        s.prepare()
        sols.append(s)
    batch = binding.Batch(sols)
    batch.step(3)
    batch.step(steps - 3)
    torch_cuda.cuda.synchronize()
    st = batch.stats()
    print(f"  stats {st}", flush=True)
    assert st["steps"] == steps
    # each member's first step runs alone, the later ones batched
    assert st["member_steps_alone"] == len(probs)
    assert st["member_steps_batched"] == len(probs) * (steps - 1)
    # a handful of launches per batched step, whatever the member count
    assert st["launches"] / (steps - 1) < 80
    for k, (s, p) in enumerate(zip(sols, probs)):
        got = _results(s, p)
        for key, ref in alone[k].items():
            assert np.array_equal(got[key], ref), (k, p.name, key,
                                                  float(np.max(np.abs(got[key] - ref))))
        stats = s.stats()
        assert stats["step"] == steps
    batch.close()
    for s in sols:
        s.close()


def test_batched_member_matches_oracle(torch_cuda, gpu_lib):
    """A torsional-plate member of a mixed batch against the FP64 oracle (FP64 form, a fixed
    iteration count so that both sides stop identically; the bars of the plate parity test)."""
    from paper_2103_06415_amd import binding
    from test_gpu_parity import fp64_tol, rel
    steps, iters = 3, 3
    p = W.plate_problem(n=32, levels=2, steps=steps)
    others = [W.cylinder_problem(n=48, steps=0), _flow_only(64, 2, 3),
              W.plate_problem(n=48, levels=1, steps=0)]
    sols = []
    for q in [p] + others:
        s = binding.Solver(q, precision=binding.IB_FP64, fixed_iters=iters)
        s.prepare()
        sols.append(s)
    batch = binding.Batch(sols)
    batch.step(steps)
    torch_cuda.cuda.synchronize()
    ora = Oracle(p, fixed_iters=iters)
    for _ in range(steps):
        ora.step()
    errs = [rel(sols[0].vorticity(g), ora.vorticity(g)) for g in range(2)]
    ef = rel(sols[0].stresses(0), ora.f)
    th = sols[0].deflection(0)
    b = ora.bodies[0][1]
    print(f"  vorticity {errs}; stresses {ef:.3e}; theta {th[0]:.6e} vs {b.theta:.6e}", flush=True)
    assert max(errs) < fp64_tol(32, steps)
    assert ef < 1e-9
    assert abs(th[0] - b.theta) < 1e-10 * max(1.0, abs(b.theta)) + 1e-14
    batch.close()
    for s in sols:
        s.close()


def test_batch_rejects_bad_members(torch_cuda, gpu_lib):
    from paper_2103_06415_amd import binding
    a = binding.Solver(W.cylinder_problem(n=32, steps=0), precision=binding.IB_FP32_FLOW)
    b = binding.Solver(W.cylinder_problem(n=32, steps=0), precision=binding.IB_FP64)
    c = binding.Solver(W.cylinder_problem(n=32, steps=0), precision=binding.IB_FP32_FLOW)
    a.prepare()
    b.prepare()
    with pytest.raises(binding.IbError) as e:
        binding.Batch([a, a])
    assert e.value.code == binding.IB_ERR_ARG
    with pytest.raises(binding.IbError) as e:
        binding.Batch([a, b])
    assert e.value.code == binding.IB_ERR_ARG
    with pytest.raises(binding.IbError) as e:
        binding.Batch([a, c])  # c is not prepared
    assert e.value.code == binding.IB_ERR_STATE
    for s in (a, b, c):
        s.close()


def test_members_step_on_alone_after_the_batch(torch_cuda, gpu_lib):
    """A batch can be destroyed and its members stepped further on their own (and a batch
    step of zero steps does nothing); the results equal a solver stepped alone throughout."""
    from paper_2103_06415_amd import binding
    probs = [W.plate_problem(n=48, levels=2, steps=0), W.cylinder_problem(n=32, steps=0)]
    ref = []
    for p in probs:
        s = binding.Solver(p, precision=binding.IB_FP32_FLOW)
        s.prepare()
        s.step(6)
        s.sync()
        ref.append((s.vorticity(0), s.stresses(0)))
        s.close()
    sols = []
    for p in probs:
        s = binding.Solver(p, precision=binding.IB_FP32_FLOW)
        s.prepare()
        sols.append(s)
    batch = binding.Batch(sols)
    batch.step(0)
    assert batch.stats()["steps"] == 0
    batch.step(4)
    batch.close()
    for s in sols:
        s.step(2)
        s.sync()
    for (w, f), s in zip(ref, sols):
        assert np.array_equal(s.vorticity(0), w)
        assert np.array_equal(s.stresses(0), f)
        assert s.stats()["step"] == 6
        s.close()


def test_a_failing_member_stops_the_batch(torch_cuda, gpu_lib):
    """A member whose body leaves its sub-domain: the batch step reports that member's error,
    says what happened, and refuses further steps (the member is marked failed)."""
    from paper_2103_06415_amd import binding
    fast = W.driven_plate_problem(n=64, levels=2, steps=0, subdomain=True)
    body = fast.bodies[0]
    # the same plate, starting near the sub-domain's right edge (x = 1.95; the plate's tip
    # at 1.825) and translating at speed 2: its tip leaves after about 13 steps of 0.005
    fast.bodies[0] = W.MovingRigid(xy_ref=body.xy_ref, ds=body.ds,
                                   motion=lambda t: (1.3 + 2.0 * t, 0.0, 0.0, 2.0, 0.0, 0.0))
    sols = []
    for p in (W.cylinder_problem(n=32, steps=0), fast):
        s = binding.Solver(p, precision=binding.IB_FP32_FLOW)
        s.prepare()
        sols.append(s)
    batch = binding.Batch(sols)
    with pytest.raises(binding.IbError) as e:
        batch.step(40)
    print(f"  batch error: {e.value}", flush=True)
    assert e.value.code == binding.IB_ERR_OUT_OF_SUBDOMAIN
    assert batch.last_error() != ""
    with pytest.raises(binding.IbError) as e2:
        batch.step(1)
    assert e2.value.code == binding.IB_ERR_STATE
    batch.close()
    for s in sols:
        s.close()


def test_large_members_equal_their_runs_alone(torch_cuda, gpu_lib):
    """Members of the 64-instance configuration whose Schur systems take the two-level
    refinement (more than 32 workgroups, shares summed in slices) next to members with the
    one-level form, in LDS size classes of their own: bit for bit their runs alone, with no
    FSI iteration continued on the host."""
    from paper_2103_06415_amd import binding
    probs = W.batch_problems()
    pick = [29, 9, 44, 7, 22]  # 756, 466, 438, 232 and 22 unknowns
    members = [probs[i] for i in pick]

    def nf(p):
        return 2 * sum(b.n if isinstance(b, W.Torsional) else len(b.xy) for b in p.bodies)

    sizes = [nf(p) for p in members]
    print(f"large members {pick}: Schur unknowns {sizes}", flush=True)
    assert max(sizes) > 700 and min(sizes) < 100
    steps = 6
    alone = []
    for k, p in zip(pick, members):
        print(f"  alone member {k} n={p.flow.n} levels={p.flow.levels}", flush=True)
        s = binding.Solver(p, precision=binding.IB_FP32_FLOW)
        s.prepare()
        s.step(steps)
        s.sync()
        alone.append(_results(s, p))
        s.close()
    sols = []
    for p in members:
        s = binding.Solver(p, precision=binding.IB_FP32_FLOW)
        s.prepare()
        sols.append(s)
    batch = binding.Batch(sols)
    batch.step(steps)
    torch_cuda.cuda.synchronize()
    st = batch.stats()
    print(f"  stats {st}", flush=True)
    assert st["fsi_resumes"] == 0
    for k, (s, p) in enumerate(zip(sols, members)):
        got = _results(s, p)
        for key, ref in alone[k].items():
            assert np.array_equal(got[key], ref), (pick[k], key,
                                                  float(np.max(np.abs(got[key] - ref))))
    batch.close()
    for s in sols:
        s.close()


def test_batched_members_that_resume_on_the_host(torch_cuda, gpu_lib):
    """Batched steps whose launched-ahead FSI iterations do not suffice for a member (it then
    continues on the host, after the control blocks were read while the batch's gated corrector
    was still queued): bit for bit the same members stepped alone."""
    from paper_2103_06415_amd import binding
    probs = [W.flag_problem(n=64, levels=3, steps=0), W.plate_problem(n=48, levels=2, steps=0)]
    steps = 12
    alone = []
    for p in probs:
        s = binding.Solver(p, precision=binding.IB_FP32_FLOW)
        s.prepare()
        s.step(steps)
        s.sync()
        alone.append(_results(s, p))
        s.close()
    sols = []
    for p in probs:
        s = binding.Solver(p, precision=binding.IB_FP32_FLOW)
        s.prepare()
        sols.append(s)
    batch = binding.Batch(sols)
    batch.step(steps)
    torch_cuda.cuda.synchronize()
    st = batch.stats()
    print(f"  stats {st}", flush=True)
    assert st["fsi_resumes"] >= 1  # the case this test is for
    for k, (s, p) in enumerate(zip(sols, probs)):
        got = _results(s, p)
        for key, ref in alone[k].items():
            assert np.array_equal(got[key], ref), (k, key, float(np.max(np.abs(got[key] - ref))))
    batch.close()
    for s in sols:
        s.close()
