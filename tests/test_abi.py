"""C-ABI checks that need no GPU: the library loads, exports every declared entry point, its
structs match the ctypes mirrors, and invalid inputs are rejected before any device work."""
import ctypes
import os
import re
import subprocess

import pytest

import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbmpwfa.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2201_05473_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2201_05473_amd import build
        build.build()
    return binding


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("lbm_init", "lbm_step", "lbm_moments", "lbm_fields", "lbm_workspace_bytes",
                     "lbm_diagnostics", "lbm_destroy", "lbm_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    so = ctypes.CDLL(lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(so, n)]
    assert not missing, missing


def test_struct_layout_matches_c(lib, tmp_path):
    """Compile a host-only probe with gcc against the header and compare offsets and sizes."""
    fields = [n for n, _ in lib.LbmConfig._fields_]
    dfields = [n for n, _ in lib.LbmDiag._fields_]
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "lbmpwfa.h"', "int main(void){",
           'printf("%zu\\n", sizeof(lbm_config));']
    src += [f'printf("%zu\\n", offsetof(lbm_config, {f}));' for f in fields]
    src += ['printf("%zu\\n", sizeof(lbm_diag));']
    src += [f'printf("%zu\\n", offsetof(lbm_diag, {f}));' for f in dfields]
    src += ["return 0;}"]
    c = tmp_path / "probe.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    expect = [ctypes.sizeof(lib.LbmConfig)] + [getattr(lib.LbmConfig, f).offset for f in fields]
    expect += [ctypes.sizeof(lib.LbmDiag)] + [getattr(lib.LbmDiag, f).offset for f in dfields]
    assert vals == expect


def test_particle_workspace_growth(lib):
    """The particle driver's workspace grows by 128 bytes per particle of capacity (two copies of
    the 7 doubles, two int32 caller indices, the re-sort's uint32 key and rank), up to the 256-byte
    rounding of its six per-particle regions."""
    base = wl.config(None, nz=64, nr=8, nb=0.3, zd0=2.0, sigma_z=0.3, sigma_r=0.2, driver=wl.PARTICLES)
    w0 = lib.lbm_workspace_bytes(dict(base, max_particles=0))
    for n in (1000, 100000):
        grow = lib.lbm_workspace_bytes(dict(base, max_particles=n)) - w0
        assert 128 * n <= grow <= 128 * n + 6 * 256, (n, grow)


@pytest.mark.parametrize("bad", [
    dict(tau=0.5), dict(tau=0.3), dict(dr=0.06), dict(c_dt_over_dz=0.6), dict(c_dt_over_dz=0.0),
    dict(nz=2), dict(nr=2), dict(ramp_kind=1, ramp_len=0.0), dict(ramp_kind=3),
    dict(periodic=1, moving_window=1), dict(periodic=2), dict(moving_window=1, c_dt_over_dz=0.3),
    dict(storage=4), dict(nb=0.1, sigma_z=0.0), dict(n_floor=-1.0), dict(check_every=-1),
    dict(collision=4), dict(collision=-1), dict(collision=1, trt_magic=0.0),
    dict(collision=1, trt_magic=float("inf")),
    dict(collision=3, mrt_sq=0.0), dict(collision=3, mrt_se=2.0), dict(collision=3, mrt_spi=float("nan")),
    dict(driver=2), dict(driver=1, max_particles=-1), dict(driver=1, max_particles=2 ** 31),
    dict(driver=1, max_particles=4, resort_every=-1),
    dict(driver=1, max_particles=4, bunch_streaming=2),
    dict(nz=8192, nr=8193), dict(nz=64, nr=65536), dict(tau=float("nan")), dict(dz=-0.05, dr=-0.05),
])
def test_invalid_configs_rejected(lib, bad):
    with pytest.raises(lib.LbmError) as ei:
        lib.lbm_workspace_bytes(wl.config(None, **bad))
    assert ei.value.code == lib.LBM_EINVAL
    assert lib.lbm_last_error() != ""


def test_largest_grid_accepted(lib):
    """2^26 sites is the largest grid (every in-plane offset stays below 2^31 elements), and 65535
    rows the most (rows are a launch dimension of some kernels)."""
    assert lib.lbm_workspace_bytes(wl.config(None, nz=8192, nr=8192, storage=wl.F64)) > 2 * 27 * 8 * 2 ** 26
    assert lib.lbm_workspace_bytes(wl.config(None, nz=64, nr=65535)) > 0


def test_trt_magic_ignored_by_other_operators(lib):
    for coll in (0, 2):
        assert lib.lbm_workspace_bytes(wl.config(None, collision=coll, trt_magic=0.0)) > 0


def test_workspace_size_scales_with_storage(lib):
    sizes = [lib.lbm_workspace_bytes(wl.config("C2", storage=s)) for s in (wl.F16, wl.F32, wl.F64)]
    assert sizes[0] < sizes[1] < sizes[2]
    # FP32: two copies of 27 populations and 6 auxiliary planes of 2048 x 512 (pitch 2048)
    assert sizes[1] >= 2 * (27 + 6) * 4 * 2048 * 512


def test_calls_without_context_fail_cleanly(lib):
    so = lib.load_library()
    assert so.lbm_step(None, 1) == lib.LBM_ESTATE
    assert so.lbm_destroy(None) == lib.LBM_ESTATE
    d = lib.LbmDiag()
    assert so.lbm_diagnostics(None, ctypes.byref(d)) == lib.LBM_ESTATE


def test_init_rejects_bad_workspace_before_device_work(lib):
    cfg = wl.config(None)
    with pytest.raises(lib.LbmError) as ei:
        lib.lbm_init(cfg, None, None, 0, 1 << 20, 0)
    assert ei.value.code == lib.LBM_EINVAL
    with pytest.raises(lib.LbmError) as ei:
        lib.lbm_init(cfg, None, None, 4096 + 8, 1 << 30, 0)   # misaligned
    assert ei.value.code == lib.LBM_EINVAL
    need = lib.lbm_workspace_bytes(cfg)
    with pytest.raises(lib.LbmError) as ei:
        lib.lbm_init(cfg, None, None, 4096, need - 256, 0)
    assert ei.value.code == lib.LBM_ENOMEM


def test_oracle_not_reachable_from_product_package():
    """The product package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2201_05473_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


def test_revolve_workspace_scales_with_snapshots(lib):
    from paper_2201_05473_amd import lbm_adjoint_revolve_workspace_bytes
    cfg = wl.config("C4")
    b1 = lbm_adjoint_revolve_workspace_bytes(cfg, 1)
    b5 = lbm_adjoint_revolve_workspace_bytes(cfg, 5)
    plane = 1024 * 256 + 64   # pitched rows, plus the 256-byte plane pad of FP32 storage
    # 27 populations, 3 moments, 3 fields and the residual word of E_r and B_theta (FP32 storage)
    state = plane * (27 * 4 + 3 * 4 + 4 * 4)
    assert b5 - b1 == 4 * state
    with pytest.raises(Exception):
        lbm_adjoint_revolve_workspace_bytes(cfg, 0)
