"""CPU-only checks of the C-ABI library: it loads, exports every entry point the
header declares, sizes workspaces and rejects invalid parameters before any
GPU work (so these run without a GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_0708_4182_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("lbm.h", "lbm_net.h")]


@pytest.fixture(scope="module")
def lib():
    from paper_0708_4182_amd import lbm
    if not os.path.exists(lbm.LIB_PATH):
        from paper_0708_4182_amd import build
        build.build()
    return lbm.load_library()


def declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lbm_init", "lbm_step", "lbm_moments", "lbm_flux"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    from paper_0708_4182_amd import lbm, net
    names = declared_functions()
    assert set(names) == set(lbm.SYMBOLS) | set(net.SYMBOLS)
    for n in names:
        assert hasattr(lib, n), n


def test_workspace_bytes(lib):
    from paper_0708_4182_amd import lbm
    p = I.Params(nx=130, ny=67)
    n32 = lbm.workspace_bytes(p)
    pitch = 192
    assert n32 >= 2 * 9 * pitch * 67 * 4 + pitch * 67 * 2
    n16 = lbm.workspace_bytes(p.replace(storage=1))
    assert n16 >= 2 * 9 * pitch * 67 * 2 and n16 < n32
    assert lbm.workspace_bytes(p.replace(nx=2)) == 0
    assert lbm.workspace_bytes(p.replace(tau=0.5)) == 0
    assert lbm.workspace_bytes(p.replace(storage=7)) == 0
    assert lbm.workspace_bytes(p.replace(rho0=0.0)) == 0
    assert lbm.workspace_bytes(p.replace(tau=float("nan"))) == 0
    assert lbm.workspace_bytes(p.replace(rho_ref=-1.0)) == 0
    assert lbm.workspace_bytes(p.replace(rho_ref=float("nan"))) == 0
    assert lbm.workspace_bytes(p.replace(rho_ref=1.8)) == n32
    # collision operator: BGK (0), TRT (1) or MRT (2) with Guo forcing, Lambda > 0 for both
    assert lbm.workspace_bytes(p.replace(collision=1)) == n32
    assert lbm.workspace_bytes(p.replace(collision=2)) == n32
    assert lbm.workspace_bytes(p.replace(collision=3)) == 0
    assert lbm.workspace_bytes(p.replace(collision=-1)) == 0
    assert lbm.workspace_bytes(p.replace(collision=1, trt_magic=0.0)) == 0
    assert lbm.workspace_bytes(p.replace(collision=1, trt_magic=float("inf"))) == 0
    assert lbm.workspace_bytes(p.replace(collision=0, trt_magic=0.0)) == n32
    # direction of the electric force: 0 (electrode) or 1 (local face normal)
    assert lbm.workspace_bytes(p.replace(elec_normal=1)) == n32
    assert lbm.workspace_bytes(p.replace(elec_normal=2)) == 0
    # rounding of 16-bit storage: 0 (nearest) or 1 (stochastic, 16-bit storage only)
    assert lbm.workspace_bytes(p.replace(storage=1, rounding=1)) == n16
    assert lbm.workspace_bytes(p.replace(storage=2, rounding=1)) == lbm.workspace_bytes(p.replace(storage=2))
    assert lbm.workspace_bytes(p.replace(storage=0, rounding=1)) == 0
    assert lbm.workspace_bytes(p.replace(storage=1, rounding=2)) == 0
    # MRT: rates of e and eps in (0, 2), unused by the other operators
    assert lbm.workspace_bytes(p.replace(collision=2)) == lbm.workspace_bytes(p.replace(collision=1))
    assert lbm.workspace_bytes(p.replace(collision=2, mrt_s_e=2.0)) == 0
    assert lbm.workspace_bytes(p.replace(collision=1, mrt_s_e=0.0, mrt_s_eps=0.0)) > 0
    # one population buffer must stay below 4 GiB (32-bit offsets)
    assert lbm.workspace_bytes(I.Params(nx=65536, ny=4096)) == 0


@pytest.mark.parametrize("bad", [dict(nx=2), dict(tau=0.4), dict(elec_walls=4),
                                 dict(elec_layers=-1), dict(storage=3), dict(rho_ref=-0.5),
                                 dict(collision=5), dict(collision=1, trt_magic=-1.0),
                                 dict(elec_normal=-1), dict(rounding=1), dict(storage=1, rounding=-1),
                                 dict(collision=2, mrt_s_e=0.0), dict(collision=2, mrt_s_eps=2.0),
                                 dict(collision=2, trt_magic=0.0)])
def test_init_rejects_invalid_params_without_gpu_work(lib, bad):
    from paper_0708_4182_amd import lbm
    import numpy as np
    p = I.Params(nx=16, ny=8).replace(**bad)
    cp = lbm.to_c_params(p)
    n = max(p.nx, 1) * p.ny
    solid = np.zeros(n, np.uint8)
    rho = np.ones(n)
    h = C.c_void_p()
    st = lib.lbm_init(C.byref(h), C.byref(cp), solid.ctypes.data_as(C.POINTER(C.c_uint8)),
                      rho.ctypes.data_as(C.POINTER(C.c_double)), None, None,
                      C.c_void_p(256), 1 << 30, None)
    assert st == -1 and not h.value
    assert lib.lbm_last_error(None)


def test_init_rejects_bad_fields_without_gpu_work(lib):
    from paper_0708_4182_amd import lbm
    import numpy as np
    p = I.Params(nx=16, ny=8)
    cp = lbm.to_c_params(p)
    h = C.c_void_p()
    args = lambda solid, rho: (C.byref(h), C.byref(cp), solid.ctypes.data_as(C.POINTER(C.c_uint8)),
                               rho.ctypes.data_as(C.POINTER(C.c_double)), None, None,
                               C.c_void_p(256), 1 << 30, None)
    rho = np.ones(128)
    rho[5] = float("nan")
    assert lib.lbm_init(*args(np.zeros(128, np.uint8), rho)) == -1
    assert b"density" in lib.lbm_last_error(None)
    assert lib.lbm_init(*args(np.ones(128, np.uint8), np.ones(128))) == -1
    assert b"no fluid" in lib.lbm_last_error(None)
    # misaligned workspace
    st = lib.lbm_init(C.byref(h), C.byref(cp), np.zeros(128, np.uint8).ctypes.data_as(C.POINTER(C.c_uint8)),
                      np.ones(128).ctypes.data_as(C.POINTER(C.c_double)), None, None,
                      C.c_void_p(4096 + 8), 1 << 30, None)
    assert st == -1
    # workspace too small
    st = lib.lbm_init(C.byref(h), C.byref(cp), np.zeros(128, np.uint8).ctypes.data_as(C.POINTER(C.c_uint8)),
                      np.ones(128).ctypes.data_as(C.POINTER(C.c_double)), None, None,
                      C.c_void_p(4096), 16, None)
    assert st == -2


def test_null_handle_calls(lib):
    assert lib.lbm_step(None, 1) == -1
    assert lib.lbm_flux(None, None, None) == -1
    assert lib.lbm_steps_done(None) == -1
    assert lib.lbm_set_kernel(None, 1) == -1
    assert lib.lbm_set_graph(None, 2) == -1
    assert lib.lbm_profile(None, None) == -1
    assert lib.lbm_get_tile(None, None, None, None) == -1
    lib.lbm_free(None)
    assert lib.lbm_status_string(-4) == b"LBM_EDIVERGED"
    assert lib.lbm_batch_set_kernel(None, 5) == -1
    assert lib.lbm_batch_get_kernel(None) == -1


def test_round_sr_validation_without_gpu_work(lib):
    # argument checks come before any HIP call; n = 0 launches nothing
    assert lib.lbm_round_sr(None, None, None, 4, 0, None) == -1      # FP32 storage has no rounding
    assert lib.lbm_round_sr(None, None, None, 4, 3, None) == -1
    assert lib.lbm_round_sr(None, None, None, -1, 1, None) == -1
    assert lib.lbm_round_sr(None, None, None, 4, 1, None) == -1      # NULL pointers with n > 0
    assert b"NULL" in lib.lbm_last_error(None)
    assert lib.lbm_round_sr(None, None, None, 0, 2, None) == 0


def test_product_path_has_no_oracle_dependency():
    """The package and the HIP sources never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_0708_4182_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "lbm_oracle" not in text and "orc_" not in text, f


def test_one_hip_runtime_in_the_process():
    """Loading the library first and torch afterwards leaves one HIP runtime
    mapped: the loader brings torch in before the library, so the library
    binds to torch's copy of the runtime instead of adding the system one."""
    import subprocess
    import sys
    code = ("from paper_0708_4182_amd import lbm; lbm.load_library(); import torch; "
            "maps = open('/proc/self/maps').read().split(chr(10)); "
            "paths = sorted({l.split()[-1] for l in maps if 'libamdhip64' in l}); "
            "print(len(paths)); print(paths)")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split()[0] == "1", out.stdout


def test_batch_workspace_validation(lib):
    from paper_0708_4182_amd import lbm
    ps = [I.Params(nx=40, ny=20), I.Params(nx=64, ny=33), I.Params(nx=300, ny=70)]
    arr = (lbm.lbm_params * 3)(*[lbm.to_c_params(p) for p in ps])
    n = lib.lbm_batch_workspace_bytes(3, arr)
    single = sum(lbm.workspace_bytes(p) for p in ps)
    assert n > 0.9 * single
    mixed = (lbm.lbm_params * 2)(lbm.to_c_params(ps[0]), lbm.to_c_params(ps[1].replace(storage=1)))
    assert lib.lbm_batch_workspace_bytes(2, mixed) == 0
    assert lib.lbm_batch_workspace_bytes(0, arr) == 0
    bad = (lbm.lbm_params * 2)(lbm.to_c_params(ps[0]), lbm.to_c_params(ps[1].replace(tau=0.3)))
    assert lib.lbm_batch_workspace_bytes(2, bad) == 0
    # one collision operator per batch
    ops = (lbm.lbm_params * 2)(lbm.to_c_params(ps[0]), lbm.to_c_params(ps[1].replace(collision=1)))
    assert lib.lbm_batch_workspace_bytes(2, ops) == 0
    trt = (lbm.lbm_params * 2)(*[lbm.to_c_params(q.replace(collision=1)) for q in ps[:2]])
    assert lib.lbm_batch_workspace_bytes(2, trt) > 0
    # one rounding per batch
    f16 = [q.replace(storage=1) for q in ps[:2]]
    rnd = (lbm.lbm_params * 2)(lbm.to_c_params(f16[0]), lbm.to_c_params(f16[1].replace(rounding=1)))
    assert lib.lbm_batch_workspace_bytes(2, rnd) == 0
    sr = (lbm.lbm_params * 2)(*[lbm.to_c_params(q.replace(rounding=1)) for q in f16])
    assert lib.lbm_batch_workspace_bytes(2, sr) > 0


def test_net_param_count_matches_the_network_definition(lib):
    """Parameter count and layout of lbm_net.h: 15 layers, W then b each."""
    from paper_0708_4182_amd import net
    import oracle.cnn as CNN
    for chans in [(32, 64, 128, 128), (12, 20, 24, 16)]:
        n = net.param_count(H=64, W=256, batch=4, chans=chans)
        assert n == CNN.param_count(CNN.layer_specs(3, 3, chans))
    assert net.param_count(H=64, W=256, batch=4) == 1209411
    assert net.param_count(H=2048, W=2048, batch=1) == 1209411     # 2^30 values in the widest layer


@pytest.mark.parametrize("bad", [dict(H=12), dict(W=4), dict(batch=0), dict(cin=0),
                                 dict(chans=(32, 0, 8, 8)), dict(batch=513), dict(chans=(32, 64, 128, 4096)),
                                 dict(cout=3000), dict(H=4096, W=2048)])
def test_net_rejects_invalid_configs_without_gpu_work(lib, bad):
    """(H=4096, W=2048: the concatenation c4 + c3 = 256 planes of one sample
    would hold 2^31 values, beyond the convolutions' 32-bit offsets.)"""
    from paper_0708_4182_amd import net
    cfg = dict(H=64, W=256, batch=2)
    cfg.update(bad)
    assert net.workspace_bytes(**cfg) == 0
    assert net.param_count(**cfg) == -1
    c = net.make_config(**cfg)
    h = C.c_void_p()
    assert lib.lbm_net_create(C.byref(h), C.byref(c), C.c_void_p(256), 1 << 30, None) == -1
    assert not h.value and lib.lbm_net_last_error(None)


def test_net_workspace_checks_without_gpu_work(lib):
    from paper_0708_4182_amd import net
    c = net.make_config(64, 256, 8)
    n = net.workspace_bytes(H=64, W=256, batch=8)
    n16 = net.workspace_bytes(H=64, W=256, batch=8, act_bf16=False)
    assert 0 < n < n16
    assert net.workspace_bytes(H=64, W=256, batch=16) > n
    h = C.c_void_p()
    assert lib.lbm_net_create(C.byref(h), C.byref(c), C.c_void_p(256 + 8), n, None) == -1
    assert lib.lbm_net_create(C.byref(h), C.byref(c), C.c_void_p(256), n - 1, None) == -2
    assert lib.lbm_net_forward(None, None, None, 1) == -1
    assert lib.lbm_net_adam(None, 1e-3, 0.9, 0.999, 1e-8) == -1
    lib.lbm_net_free(None)


def test_bench_traffic_lookup(tmp_path, monkeypatch):
    """bench.py reports counter traffic only for a record of the current kernel
    source and the timed tile; records in either layout (one per storage, or a
    list per storage) are read, and stale or foreign ones give None."""
    import json
    import sys
    sys.path.insert(0, ROOT)
    import bench
    sha = bench.kernel_sha()
    table = {"f32": [{"kernel_sha": sha, "tile": [512, 0, "fused8"], "bytes_per_launch": 123},
                     {"kernel_sha": "0" * 16, "tile": [512, 64, "fused"], "bytes_per_launch": 7}],
             "f16": {"kernel_sha": sha, "tile": [512, 0, "fused"], "bytes_per_launch": 45},
             "_note": "text"}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(table))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("f32", [512, 0, "fused8"]) == 123
    assert bench.measured_traffic("f32", [512, 64, "fused"]) is None      # another kernel source
    assert bench.measured_traffic("f32", [256, 0, "fused8"]) is None      # another tile
    assert bench.measured_traffic("f16", (512, 0, "fused")) == 45
    assert bench.measured_traffic("bf16", [512, 0, "fused"]) is None


def test_bench_roofline_per_launch(monkeypatch):
    """The bench's HBM roofline charges each launch its algorithmic bytes
    (18 values per fluid node, read once and written once): a two-step launch
    covers two time steps with the bytes of one, so its achieved rate is half
    the single-step equivalent, which is reported beside it."""
    import bench
    monkeypatch.setattr(bench, "measured_traffic", lambda name, tile: None)
    nsites, nfluid = 1000, 800
    one = bench.step_line("f32", {"step_ms": 0.001, "tile": [256, 64, "fused"]}, nsites, nfluid)
    two = bench.step_line("f32", {"step_ms": 0.001, "tile": [512, 137, "two"]}, nsites, nfluid)
    half = bench.step_line("f16", {"step_ms": 0.001, "tile": [256, 67, "two"]}, nsites, nfluid)
    assert one["roofline"]["achieved"] == round(72 * 800 / 1e-6 / 1e9, 1)
    assert one["roofline"]["steps_per_launch"] == 1 and "single_step_equivalent" not in one["roofline"]
    assert two["roofline"]["steps_per_launch"] == 2 and two["roofline"]["launch_ms"] == 0.002
    assert two["roofline"]["achieved"] == round(one["roofline"]["achieved"] / 2, 1)
    assert two["roofline"]["single_step_equivalent"]["GB/s"] == one["roofline"]["achieved"]
    assert half["roofline"]["achieved"] == round(36 * 800 / 2e-6 / 1e9, 1)
    assert one["mlups"] == two["mlups"] == round(nsites / 1e-6 / 1e6, 1)


def test_bench_batch_line_per_launch():
    """The batch line charges a launch of the sweep table the bytes of one step
    (each population read and written once per launch), so at two steps per
    launch its achieved rate is half the single-step equivalent."""
    import bench
    bt = {"kernel": "two", "tile": [256, 32], "mlups": 1.0, "ms_per_step": 0.5, "achieved_GBs": 4000.0}
    two = bench.batch_line(bt)
    one = bench.batch_line(dict(bt, kernel="fused"))
    three = bench.batch_line(dict(bt, kernel="three"))
    assert one["roofline"]["achieved"] == 4000.0 and "single_step_equivalent" not in one["roofline"]
    assert two["roofline"]["achieved"] == 2000.0 and two["roofline"]["steps_per_launch"] == 2
    assert two["roofline"]["single_step_equivalent"] == {"GB/s": 4000.0, "frac": 0.5}
    assert three["roofline"]["frac"] == round(4000.0 / 3 / 8000.0, 4)
    assert two["kernel"] == "two" and two["tile"] == [256, 32]
