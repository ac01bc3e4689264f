"""The C-ABI library loads and exports every entry point its header declares (CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ibfsi.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ib_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2103_06415_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2103_06415_amd import build
        build.build()
    return binding.load()


def test_header_declares_the_step_api():
    syms = declared_symbols()
    for name in ("ib_create", "ib_add_rigid", "ib_add_torsional", "ib_add_deformable",
                 "ib_set_subdomain", "ib_set_vorticity", "ib_prepare", "ib_step", "ib_sync",
                 "ib_read_stresses", "ib_read_deflection", "ib_read_vorticity", "ib_destroy",
                 "ib_status_str", "ib_op_solve"):
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(os.path.join(ROOT, "paper_2103_06415_amd", "lib", "libibfsi.so"))
    missing = [s for s in declared_symbols() if not hasattr(raw, s)]
    assert not missing, missing


def test_status_strings(lib):
    assert lib.ib_status_str(0) == b"ok"
    assert b"sub-domain" in lib.ib_status_str(-6)
    assert lib.ib_status_str(-100) == b"unknown status"


def test_create_rejects_bad_configs_without_a_gpu(lib):
    from paper_2103_06415_amd import binding
    out = ctypes.c_void_p()
    for n, levels, h in ((100, 1, 0.1), (32, 0, 0.1), (32, 1, -1.0), (30, 1, 0.1)):
        cfg = binding.IbConfig(n=n, levels=levels, h=h, re=100.0, dt=0.01)
        assert lib.ib_create(ctypes.byref(cfg), None, None, ctypes.byref(out)) == -1
    assert lib.ib_create(None, None, None, ctypes.byref(out)) == -1


def test_null_handles_are_rejected(lib):
    assert lib.ib_prepare(None) == -1
    assert lib.ib_step(None, 1) == -1
    assert lib.ib_destroy(None) == -1


def test_batch_entry_points_reject_bad_arguments(lib):
    import ctypes
    out = ctypes.c_void_p()
    assert lib.ib_batch_create(None, 1, None, ctypes.byref(out)) == -1
    members = (ctypes.c_void_p * 2)(None, None)
    assert lib.ib_batch_create(members, 2, None, ctypes.byref(out)) == -1
    assert lib.ib_batch_create(members, 0, None, ctypes.byref(out)) == -1
    assert not out.value
    assert lib.ib_batch_step(None, 1) == -1
    assert lib.ib_batch_destroy(None) == -1
    assert lib.ib_batch_last_error(None) == b"null batch"


def _config(binding, n, levels):
    return binding.IbConfig(n=n, levels=levels, h=2.0 / n, re=200.0, dt=0.4 / n, cx=0.0, cy=0.0,
                            precision=binding.IB_FP32_FLOW, newton_tol=1e-7, newton_max_iter=20,
                            drop_tol=0.007)


def test_create_allocates_nothing_and_estimates_memory(lib):
    """ib_create holds no device memory (so it works without a GPU); the admission
    estimate grows with the grid, the levels and the precision."""
    from paper_2103_06415_amd import binding
    est = {}
    for n, levels, prec in ((64, 1, binding.IB_FP32_FLOW), (128, 1, binding.IB_FP32_FLOW),
                            (128, 3, binding.IB_FP32_FLOW), (128, 3, binding.IB_FP64)):
        cfg = _config(binding, n, levels)
        cfg.precision = prec
        h = ctypes.c_void_p()
        assert lib.ib_create(ctypes.byref(cfg), None, None, ctypes.byref(h)) == 0
        res, peak = ctypes.c_int64(), ctypes.c_int64()
        assert lib.ib_estimate_bytes(h, ctypes.byref(res), ctypes.byref(peak)) == 0
        assert 0 < res.value <= peak.value
        est[(n, levels, prec)] = res.value
        out = (ctypes.c_double * ((n - 1) * (n - 1)))()
        assert lib.ib_read_vorticity(h, 0, out, (n - 1) * (n - 1)) == -2  # nothing on the device yet
        assert lib.ib_release(h) == 0
        assert lib.ib_destroy(h) == 0
    f32, f64 = binding.IB_FP32_FLOW, binding.IB_FP64
    assert est[(64, 1, f32)] < est[(128, 1, f32)] < est[(128, 3, f32)] < est[(128, 3, f64)]
    # one FP32 level of n^2 cells holds about 6 arrays of n^2 floats (state, history,
    # work): the estimate is of that order, not wildly off
    n2 = 128 * 128 * 4
    assert 3 * n2 < est[(128, 1, f32)] < 40 * n2


def test_estimate_counts_the_subdomain_operator(lib):
    from paper_2103_06415_amd import binding
    cfg = _config(binding, 128, 2)
    h = ctypes.c_void_p()
    assert lib.ib_create(ctypes.byref(cfg), None, None, ctypes.byref(h)) == 0
    bid = ctypes.c_int32()
    assert lib.ib_add_torsional(h, 11, 0.0, 0.0, 0.5, -0.3, 5.0, 1.0, 0.1, 0.0, 0.0,
                                ctypes.byref(bid)) == 0
    r0, p0 = ctypes.c_int64(), ctypes.c_int64()
    assert lib.ib_estimate_bytes(h, ctypes.byref(r0), ctypes.byref(p0)) == 0
    assert lib.ib_set_subdomain(h, -0.05, 0.55, -0.4, 0.4) == 0
    r1, p1 = ctypes.c_int64(), ctypes.c_int64()
    assert lib.ib_estimate_bytes(h, ctypes.byref(r1), ctypes.byref(p1)) == 0
    rows = 2 * (int(0.6 / cfg.h) + 3) * (int(0.8 / cfg.h) + 3)
    assert r1.value - r0.value >= rows * 800 * 12
    assert lib.ib_destroy(h) == 0


def test_operator_import_validates_its_input(lib):
    from paper_2103_06415_amd import binding
    cfg = _config(binding, 64, 1)
    h = ctypes.c_void_p()
    assert lib.ib_create(ctypes.byref(cfg), None, None, ctypes.byref(h)) == 0
    bad = b"NOTANOP!" + bytes(32)
    assert lib.ib_import_operator(h, bad, len(bad)) == -1
    good_header = b"IBOP0001" + (1).to_bytes(8, "little") + (0).to_bytes(24, "little") + bytes(8)
    assert lib.ib_import_operator(h, good_header, len(good_header)) == 0
    assert lib.ib_import_operator(h, good_header, len(good_header) - 1) == -1
    used = ctypes.c_int64()
    assert lib.ib_export_operator(h, None, 0, ctypes.byref(used)) == -2  # nothing built yet
    assert lib.ib_set_operator_cache(-1) == -1
    assert lib.ib_destroy(h) == 0


def test_flow_variant_table_and_forcing(lib):
    """The transform-kernel configurations are listed, and forcing one is validated: only
    single precision at the measured sizes has alternatives to configuration 0; the row
    kernels have 8 configurations, the column solve 9, the last of them (register-resident
    transforms, FFT split 32) at n = 1024 only."""
    from paper_2103_06415_amd import binding
    counts = {0: 8, 1: 9}
    for kind in (0, 1):
        seen = set()
        for v in range(counts[kind]):
            w, t, r = binding.flow_variant_info(kind, v)
            assert w >= 1 and t in (64, 128, 256, 512, 1024) and r in (4, 8, 16, 32)
            assert t % 64 == 0 and t >= 2 * w
            seen.add((w, t, r))
        assert len(seen) == counts[kind]  # all distinct
    assert binding.flow_variant_info(1, 8) == (4, 128, 32)
    w, t, r = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert lib.ib_flow_variant_info(2, 0, ctypes.byref(w), ctypes.byref(t), ctypes.byref(r)) == -1
    assert lib.ib_flow_variant_info(0, 8, ctypes.byref(w), ctypes.byref(t), ctypes.byref(r)) == -1
    assert lib.ib_flow_variant_info(1, 9, ctypes.byref(w), ctypes.byref(t), ctypes.byref(r)) == -1
    for n, prec, ok in ((256, binding.IB_FP32_FLOW, True), (128, binding.IB_FP32_FLOW, False),
                        (256, binding.IB_FP64, False)):
        cfg = _config(binding, n, 1)
        cfg.precision = prec
        h = ctypes.c_void_p()
        assert lib.ib_create(ctypes.byref(cfg), None, None, ctypes.byref(h)) == 0
        assert lib.ib_set_flow_variants(h, 0, 0, 0) == 0  # defaults are always allowed
        assert lib.ib_set_flow_variants(h, 1, 2, 3) == (0 if ok else -1)
        assert lib.ib_set_flow_variants(h, 0, 9, 0) == -1
        assert lib.ib_set_flow_variants(h, 8, 0, 0) == -1     # rows: 8 configurations
        assert lib.ib_set_flow_variants(h, 0, 8, 0) == -1     # column 8: n = 1024 only
        tun = binding.IbFlowTuning()
        assert lib.ib_get_flow_tuning(h, ctypes.byref(tun)) == 0
        if ok:
            assert (tun.rhs_variant, tun.col_variant, tun.idst_variant) == (1, 2, 3)
            assert lib.ib_set_flow_variants(h, -1, 5, -1) == 0
            assert lib.ib_get_flow_tuning(h, ctypes.byref(tun)) == 0
            assert (tun.rhs_variant, tun.col_variant, tun.idst_variant) == (1, 5, 3)
        assert lib.ib_destroy(h) == 0


def test_rectangular_levels_are_validated_and_estimated(lib):
    """ny (cells along y) takes the same sizes as n (2000 and 4000 included, 4000 in single
    precision only); the matrix-core transform form stays square; the memory estimate follows
    nx x ny."""
    from paper_2103_06415_amd import binding
    est = {}
    for n, ny, prec, ok in ((64, 32, binding.IB_FP32_FLOW, True), (64, 30, binding.IB_FP32_FLOW, False),
                            (64, 0, binding.IB_FP32_FLOW, True), (64, 128, binding.IB_FP64, True),
                            (64, 32, binding.IB_FP32_FLOW_BF16_DST, False), (64, -4, binding.IB_FP64, False),
                            (64, 2000, binding.IB_FP64, True), (64, 4000, binding.IB_FP32_FLOW, True),
                            (64, 4000, binding.IB_FP64, False), (64, 3000, binding.IB_FP32_FLOW, False),
                            (4000, 2000, binding.IB_FP32_FLOW, True)):
        cfg = _config(binding, n, 2)
        cfg.h = 4.0 / n
        cfg.ny = ny
        cfg.precision = prec
        h = ctypes.c_void_p()
        rc = lib.ib_create(ctypes.byref(cfg), None, None, ctypes.byref(h))
        assert rc == (0 if ok else -1), (n, ny, prec, rc)
        if ok:
            res, peak = ctypes.c_int64(), ctypes.c_int64()
            assert lib.ib_estimate_bytes(h, ctypes.byref(res), ctypes.byref(peak)) == 0
            est[(ny, prec)] = res.value
            assert lib.ib_destroy(h) == 0
    assert est[(32, binding.IB_FP32_FLOW)] < est[(0, binding.IB_FP32_FLOW)]
