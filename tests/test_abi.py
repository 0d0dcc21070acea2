"""The C-ABI library loads, exports every function include/pba.h declares, and the binding's
structs have the header's layout.  No GPU call is made."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2303_16878_amd as pba

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pba.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pba_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = pba.load_library()
    names = _declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(pba.ABI_FUNCTIONS) == names
    out = subprocess.run(["nm", "-D", "--defined-only", pba.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (pba_\w+)", out))
    assert set(names) <= exported


def test_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "pba.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\\n", sizeof(pba_sensor), sizeof(pba_config), sizeof(pba_eval_out),
         sizeof(pba_iter_log), sizeof(pba_timings));
  printf("%zu %zu %zu %zu\\n", offsetof(pba_config, stream), offsetof(pba_config, occlusion_tau_spherical),
         offsetof(pba_sensor, offset), offsetof(pba_eval_out, pair_out));
  printf("%d\\n", PBA_PAIR_OUT_LEN);
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    lines = subprocess.check_output([str(exe)], text=True).split("\n")
    sizes = [int(v) for v in lines[0].split()]
    assert sizes == [ctypes.sizeof(pba.pba_sensor), ctypes.sizeof(pba.pba_config), ctypes.sizeof(pba.pba_eval_out),
                     ctypes.sizeof(pba.pba_iter_log), ctypes.sizeof(pba.pba_timings)]
    offs = [int(v) for v in lines[1].split()]
    assert offs == [pba.pba_config.stream.offset, pba.pba_config.occlusion_tau_spherical.offset, pba.pba_sensor.offset.offset,
                    pba.pba_eval_out.pair_out.offset]
    assert int(lines[2]) == pba.PBA_PAIR_OUT_LEN


def test_config_defaults_and_status_strings():
    cfg = pba.config_default()
    assert cfg.precision == pba.PBA_F32 and cfg.channels == 5 and cfg.huber_delta == 0.1
    assert cfg.occlusion_tau_pinhole == 0.5 and cfg.occlusion_tau_spherical == 1.0
    lib = pba.load_library()
    assert lib.pba_status_string(pba.PBA_EINVAL) == b"invalid argument"
    assert lib.pba_status_string(123) == b"unknown status"


def test_invalid_config_rejected_before_any_device_call():
    lib = pba.load_library()
    cfg = pba.config_default()
    cfg.channels = 3
    h = ctypes.c_void_p()
    assert lib.pba_create(ctypes.byref(cfg), ctypes.byref(h)) == pba.PBA_EINVAL
    cfg = pba.config_default()
    cfg.occlusion_tau_spherical = -1.0
    assert lib.pba_create(ctypes.byref(cfg), ctypes.byref(h)) == pba.PBA_EINVAL


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    monkeypatch.setattr(pba, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        pba.load_library(str(tmp_path / "nope.so"))


def test_product_ate_matches_oracle_alignment():
    """The library's trajectory metric (orthonormal-matrix form) agrees with the oracle's
    quaternion form of Horn's alignment."""
    import numpy as np
    import oracle
    from paper_2303_16878_amd.metrics import ate_rmse
    rng = np.random.default_rng(5)
    for _ in range(5):
        A = np.zeros((30, 12))
        A[:, 9:] = rng.normal(size=(30, 3)) * 10
        B = A.copy()
        B[:, 9:] = A[:, 9:] @ np.linalg.qr(rng.normal(size=(3, 3)))[0].T + rng.normal(size=(30, 3)) * 0.1
        assert abs(ate_rmse(A, B) - oracle.ate_rmse(A, B)) < 1e-12
