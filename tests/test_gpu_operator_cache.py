"""Offline operator reuse: cached and imported operators give the same steps as a built one."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(problem, steps, prec, data=None):
    from paper_2103_06415_amd import binding
    s = binding.Solver(problem, precision=prec, torch_alloc=False)
    if data is not None:
        s.import_operator(data)
    s.prepare()
    s.step(steps)
    s.sync()
    out = {"vort": s.vorticity(0), "f": s.stresses(0), "d": s.deflection(0),
           "source": s.stats()["operator_source"], "nnz": s.stats()["subdomain_nnz"]}
    return s, out


@pytest.mark.parametrize("which", ["plate", "flag", "cylinder"])
def test_cached_and_imported_operators(torch_cuda, gpu_lib, which):
    from paper_2103_06415_amd import binding
    make = {"plate": lambda: W.plate_problem(n=32, levels=2, steps=4),
            "flag": lambda: W.flag_problem(n=32, levels=2, steps=4),
            "cylinder": lambda: W.cylinder_problem(n=32, steps=4)}[which]
    print(f"operator cache {which}", flush=True)
    binding.set_operator_cache(0)           # empty
    binding.set_operator_cache(1 << 33)
    a, ra = _run(make(), 4, binding.IB_FP64)
    b, rb = _run(make(), 4, binding.IB_FP64)
    assert ra["source"] == 0 and rb["source"] == 1
    data = a.export_operator()
    binding.set_operator_cache(0)
    c, rc = _run(make(), 4, binding.IB_FP64, data)
    assert rc["source"] == 2
    for r in (rb, rc):
        assert r["nnz"] == ra["nnz"]
        for key in ("vort", "f", "d"):
            assert np.array_equal(r[key], ra[key]), key
    for s in (a, b, c):
        s.close()
    binding.set_operator_cache(1 << 33)


def test_import_of_a_foreign_operator_is_rejected(torch_cuda, gpu_lib):
    from paper_2103_06415_amd import binding
    binding.set_operator_cache(0)
    a, _ = _run(W.plate_problem(n=32, levels=2, steps=1), 1, binding.IB_FP64)
    data = a.export_operator()
    a.close()
    p = W.plate_problem(n=32, levels=2, steps=1)
    p.subdomain = (p.subdomain[0], p.subdomain[1] + 0.1, p.subdomain[2], p.subdomain[3])
    s = binding.Solver(p, precision=binding.IB_FP64, torch_alloc=False)
    s.import_operator(data)
    with pytest.raises(binding.IbError) as e:
        s.prepare()
    assert e.value.code == -1
    s.close()
    binding.set_operator_cache(1 << 33)
