"""Host-side checks of the C ABI that need no GPU: the built library loads,
exports every function include/lbm.h declares, validates parameter sets and
refuses to run without a gfx950 device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")
MLP_HEADER = os.path.join(ROOT, "include", "mlp.h")
HEADER3 = os.path.join(ROOT, "include", "lbm3d.h")
LIB = os.path.join(ROOT, "paper_2609_26332_amd", "liblbm_hip.so")


def declared_functions(header=HEADER, prefix="lbm_"):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(" + prefix + r"[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lbm():
    if not os.path.exists(LIB):
        pytest.fail("liblbm_hip.so is not built; run __graft_entry__.build()")
    from paper_2609_26332_amd import lbm as binding

    return binding


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("lbm_init", "lbm_step", "lbm_reduce_invariants", "lbm_fetch_fields", "lbm_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol(lbm):
    L = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(L, name), name
    assert sorted(lbm.EXPORTS) == declared_functions()
    from paper_2609_26332_amd import surrogate
    mlp_names = declared_functions(MLP_HEADER, "mlp_")
    assert sorted(surrogate.EXPORTS) == mlp_names
    for name in mlp_names:
        assert hasattr(L, name), name
    assert L.mlp_param_count() == 133634
    from paper_2609_26332_amd import lbm3d
    names3 = declared_functions(HEADER3, "lbm3d_")
    assert sorted(lbm3d.EXPORTS) == names3
    for name in names3:
        assert hasattr(L, name), name


def test_3d_parameter_validation_without_a_device(lbm):
    """lbm3d_required_bytes validates a parameter set on the host."""
    from paper_2609_26332_amd import inputs, lbm3d

    L = lbm3d.lib()
    n = ctypes.c_size_t()
    p = lbm3d.make_params(inputs.drop3d(16, 5.0), lbm.FP64)
    assert L.lbm3d_required_bytes(ctypes.byref(p), ctypes.byref(n)) == 0 and n.value > 57 * 2 * 16 ** 3 * 8
    bad = lbm3d.make_params(dict(inputs.drop3d(16, 5.0), nz=2), lbm.FP64)
    assert L.lbm3d_required_bytes(ctypes.byref(bad), ctypes.byref(n)) == lbm.LbmError(-1, "").code
    assert b"nz" in L.lbm3d_last_error(None)
    bad = lbm3d.make_params(inputs.drop3d(16, 5.0), lbm.FP16_SHIFTED)
    assert L.lbm3d_required_bytes(ctypes.byref(bad), ctypes.byref(n)) == -1
    # the kernels address a node's values with 32-bit byte offsets: 2^29 nodes or more are refused
    big = lbm3d.make_params(dict(inputs.drop3d(16, 5.0), nx=1024, ny=1024, nz=512), lbm.FP32)
    assert L.lbm3d_required_bytes(ctypes.byref(big), ctypes.byref(n)) == -1
    assert b"2^29" in L.lbm3d_last_error(None)
    ok = lbm3d.make_params(dict(inputs.drop3d(16, 5.0), nx=1024, ny=1024, nz=511), lbm.FP32)
    assert L.lbm3d_required_bytes(ctypes.byref(ok), ctypes.byref(n)) == 0


def test_param_struct_layout_matches_header(lbm):
    # 10 int32 (40 bytes) then doubles: the binding must agree with the header
    text = open(HEADER).read()
    body = text[text.index("typedef struct {", text.index("LBM_INIT_BUBBLE")):text.index("} lbm_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    n_int = sum(len(re.findall(r"[a-z_0-9]+(?:\[\d+\])?", decl.split(None, 1)[1]))
                for decl in re.findall(r"int32_t[^;]+;", body))
    n_dbl = 0
    for decl in re.findall(r"double[^;]+;", body):
        for item in decl[len("double"):].strip(" ;").split(","):
            m = re.search(r"\[(\d+)\]", item)
            n_dbl += int(m.group(1)) if m else 1
    assert ctypes.sizeof(lbm.Params) == 4 * n_int + 8 * n_dbl
    assert lbm.Params.sigma_gl0.offset == 4 * n_int


def test_required_bytes_and_validation(lbm):
    from paper_2609_26332_amd import inputs

    cfg = inputs.stationary_drop()
    n64 = lbm.required_bytes(cfg, "fp64")
    n32 = lbm.required_bytes(cfg, "fp32")
    N = 64 * 64
    assert n64 > 2 * 27 * N * 8 and n32 > 2 * 27 * N * 4 and n64 > n32
    bad = [dict(cfg, nx=2), dict(cfg, psi_b=1.0), dict(cfg, bc_bottom=inputs.WALL_WET), dict(cfg, tile_rows=5),
           dict(cfg, s_g=[1, 2.5, 1, 1, 1]), dict(cfg, sigma_gl0=0.0)]
    wet = inputs.sessile_drop(nx=32, ny=16, R=5)
    bad.append(dict(wet, theta0_deg=0.0))
    bad.append(dict(wet, lambda_s=0.0))  # adsorbing wall needs lambda_s > 0
    for b in bad:
        with pytest.raises(lbm.LbmError) as e:
            lbm.required_bytes(b, "fp64")
        assert e.value.code == -1


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU is present")
def test_init_without_device_reports_device_error(lbm):
    from paper_2609_26332_amd import inputs

    p = lbm.make_params(inputs.stationary_drop(nx=16, ny=16, R=4), lbm.FP64)
    h = ctypes.c_void_p()
    rc = lbm.lib().lbm_init(ctypes.byref(p), None, 0, None, ctypes.byref(h))
    assert rc == -4 and not h.value
    assert b"device" in lbm.lib().lbm_last_error(None).lower()


def test_batch_validation(lbm):
    """Batch argument checks happen on the host (no device needed)."""
    import ctypes

    from paper_2609_26332_amd import inputs

    wall = inputs.sessile_drop(nx=64, ny=32, R=10.0)
    per = inputs.stationary_drop(nx=32, ny=32, R=8.0)
    L = lbm.lib()
    n = ctypes.c_size_t()
    arr = (lbm.Params * 2)(lbm.make_params(wall, lbm.FP32), lbm.make_params(per, lbm.FP32))
    assert L.lbm_batch_required_bytes(arr, 2, ctypes.byref(n)) == -1
    assert b"periodic" in L.lbm_batch_last_error(None)
    arr = (lbm.Params * 2)(lbm.make_params(wall, lbm.FP32), lbm.make_params(wall, lbm.FP64))
    assert L.lbm_batch_required_bytes(arr, 2, ctypes.byref(n)) == -1
    arr = (lbm.Params * 2)(lbm.make_params(wall, lbm.FP32), lbm.make_params(dict(wall, nx=2), lbm.FP32))
    assert L.lbm_batch_required_bytes(arr, 2, ctypes.byref(n)) == -1
    assert b"case 1" in L.lbm_batch_last_error(None)
    arr = (lbm.Params * 2)(lbm.make_params(wall, lbm.FP32), lbm.make_params(dict(wall, nx=96, ny=48, R0=14.0), lbm.FP32))
    assert L.lbm_batch_required_bytes(arr, 2, ctypes.byref(n)) == 0
    single = ctypes.c_size_t()
    assert L.lbm_required_bytes(ctypes.byref(arr[0]), ctypes.byref(single)) == 0
    assert n.value > single.value
    assert L.lbm_batch_required_bytes(arr, 0, ctypes.byref(n)) == -1
    # the accuracy test of Sec. 4.1 runs on single handles only, and only as specified
    mms = inputs.manufactured(32)
    arr = (lbm.Params * 2)(lbm.make_params(mms, lbm.FP64), lbm.make_params(mms, lbm.FP64))
    assert L.lbm_batch_required_bytes(arr, 2, ctypes.byref(n)) == -1
    assert b"accuracy test" in L.lbm_batch_last_error(None)
    assert L.lbm_required_bytes(ctypes.byref(arr[0]), ctypes.byref(single)) == 0
    for bad in (lbm.make_params(mms, lbm.FP32), lbm.make_params(dict(mms, nx=33), lbm.FP64),
                lbm.make_params(dict(mms, constraint_phi=inputs.NONLINEAR), lbm.FP64)):
        assert L.lbm_required_bytes(ctypes.byref(bad), ctypes.byref(single)) == -1
        assert b"accuracy test" in L.lbm_last_error(None)
    # the autotuner and its report refuse missing arguments before touching a device
    i32 = ctypes.c_int32()
    assert L.lbm_batch_autotune(None, 4, ctypes.byref(i32)) == -1
    assert L.lbm_batch_autotune_report(None, 0, None, None, None, None, ctypes.byref(i32)) == -1
    assert b"null" in L.lbm_batch_last_error(None)
