"""CPU checks of the C ABI: the library loads, exports every entry point that
include/mhd.h declares, its structs match the binding's ctypes layout, and
argument validation happens before any device call (no GPU needed)."""
import os
import re
import subprocess

import pytest

from paper_2606_12753_amd import build as hb
from paper_2606_12753_amd import mhd
from paper_2606_12753_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mhd.h")


@pytest.fixture(scope="module")
def lib():
    if hb.stale():
        hb.build()
    return mhd.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mhd_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert set(names) == set(mhd.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", hb.LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (mhd_[a-z_]+)", out))
    for n in names:
        assert n in exported, n
        assert hasattr(lib, n)


def test_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(f'''
#include <stdio.h>
#include <stddef.h>
#include "{HEADER}"
int main(void) {{
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(mhd_box), offsetof(mhd_box, lo),
         offsetof(mhd_box, bc_lo), offsetof(mhd_box, gamma), sizeof(mhd_config),
         offsetof(mhd_config, stream), offsetof(mhd_config, flags),
         offsetof(mhd_config, rk_stages), offsetof(mhd_config, riemann),
         offsetof(mhd_config, recon), offsetof(mhd_config, ct_emf),
         offsetof(mhd_config, limiter));
  return 0;
}}''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-o", str(exe), str(prog)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    import ctypes as C
    got = [C.sizeof(mhd.mhd_box), mhd.mhd_box.lo.offset, mhd.mhd_box.bc_lo.offset,
           mhd.mhd_box.gamma.offset, C.sizeof(mhd.mhd_config), mhd.mhd_config.stream.offset,
           mhd.mhd_config.flags.offset, mhd.mhd_config.rk_stages.offset,
           mhd.mhd_config.riemann.offset, mhd.mhd_config.recon.offset,
           mhd.mhd_config.ct_emf.offset, mhd.mhd_config.limiter.offset]
    assert vals == got


def test_validation_before_device(lib):
    good = W.BoxSpec((8, 8, 8))
    nbytes = mhd.mhd_workspace_bytes([good])
    assert nbytes > 8 * 8 * 8 * 8 * 16
    bad_cases = [
        W.BoxSpec((0, 8, 8)),
        W.BoxSpec((8, 8, 8), hi=(1.0, 0.0, 1.0)),
        W.BoxSpec((8, 8, 8), gamma=1.0),
        W.BoxSpec((8, 8, 8), cfl=0.0),
        W.BoxSpec((8, 8, 8), bc=(0, 2, 0)),
        W.BoxSpec((1, 1, 1)),                    # no active axis: dt undefined
        W.BoxSpec(((1 << 20) + 1, 2, 1)),        # axis longer than 2^20 cells
        W.BoxSpec((1024, 1024, 513)),            # more than 2^29 cells
        W.BoxSpec((1024, 1024, 512), bc=(1, 0, 0)),  # 2^29 cells, more face positions
    ]
    for spec in bad_cases:
        with pytest.raises(mhd.MhdError) as ei:
            mhd.mhd_workspace_bytes([spec])
        assert ei.value.code == mhd.MHD_E_INVAL
        with pytest.raises(mhd.MhdError) as ei:
            mhd.Sim([spec])
        assert ei.value.code == mhd.MHD_E_INVAL
    with pytest.raises(mhd.MhdError) as ei:
        mhd.mhd_workspace_bytes([good], precision=7)
    assert ei.value.code == mhd.MHD_E_INVAL
    with pytest.raises(mhd.MhdError) as ei:
        mhd.mhd_workspace_bytes([])
    assert ei.value.code == mhd.MHD_E_INVAL
    for kw in ({"rk": 4}, {"solver": 2}, {"recon": 2}, {"emf": 4}, {"emf": -1}, {"limiter": 3}):
        with pytest.raises(mhd.MhdError) as ei:
            mhd.mhd_workspace_bytes([good], **kw)
        assert ei.value.code == mhd.MHD_E_INVAL, kw
    assert mhd.mhd_workspace_bytes([good], solver="hll") == nbytes
    # the upwind CT keeps the outer wave speeds of every face: two more face
    # arrays per axis, in the arithmetic type of the path
    uct = mhd.mhd_workspace_bytes([good], emf="uct_hll")
    assert uct > nbytes
    assert mhd.mhd_workspace_bytes([good], emf="uct_hll", precision=mhd.MHD_MIXED) < uct
    # the largest accepted box: 2^29 cells (periodic), and one active axis
    big = mhd.mhd_workspace_bytes([W.BoxSpec((1024, 1024, 512))])
    assert big > (1 << 29) * 8 * 16
    assert mhd.mhd_workspace_bytes([W.BoxSpec((1, 1, 7))]) > 0


def test_workspace_grows_with_precision_and_boxes(lib):
    a = mhd.mhd_workspace_bytes([W.BoxSpec((16, 16, 16))], precision=mhd.MHD_FP64)
    b = mhd.mhd_workspace_bytes([W.BoxSpec((16, 16, 16))], precision=mhd.MHD_MIXED)
    c = mhd.mhd_workspace_bytes([W.BoxSpec((16, 16, 16))] * 3, precision=mhd.MHD_FP64)
    assert b < a < c


def test_create_without_gpu_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(mhd.MhdError) as ei:
        mhd.Sim([W.BoxSpec((8, 8, 8))])
    assert ei.value.code == mhd.MHD_E_DEVICE


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(mhd, "_LIB", None)
    monkeypatch.setattr(hb, "LIB", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        mhd.load()


def test_dt_noalloc_rejects_before_device_work(lib):
    """The allocation-free time-step query validates on the host: a box
    beyond its scratch capacity (2^28 cells), a bad box and NULL arrays are
    rejected with MHD_E_INVAL without touching a device."""
    import ctypes as C
    null5 = (C.c_void_p * 5)()
    null3 = (C.c_void_p * 3)()
    big = mhd._box_struct(W.BoxSpec((1024, 1024, 257)))
    assert lib.mhd_dt_noalloc(C.byref(big), null5, null3, 0.0, None, None) == mhd.MHD_E_INVAL
    assert b"scratch capacity" in lib.mhd_last_error(None)
    bad = mhd._box_struct(W.BoxSpec((8, 8, 8), gamma=0.5))
    assert lib.mhd_dt_noalloc(C.byref(bad), null5, null3, 0.0, None, None) == mhd.MHD_E_INVAL
    ok = mhd._box_struct(W.BoxSpec((8, 8, 8)))
    assert lib.mhd_dt_noalloc(C.byref(ok), null5, null3, 0.0, None, None) == mhd.MHD_E_INVAL
    assert b"NULL" in lib.mhd_last_error(None)
    assert lib.mhd_dt_noalloc(None, null5, null3, 0.0, None, None) == mhd.MHD_E_INVAL
