"""The C-ABI library loads, exports every declared entry point, and rejects bad arguments on the host."""
import ctypes
import os
import re

import pytest

import paper_2407_06042_amd as dm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dmala.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dmala_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = dm.lib()
    names = _declared()
    assert set(names) == set(dm.EXPORTED)
    for n in names:
        assert hasattr(L, n), n
    assert b"gfx950" in L.dmala_version()


def test_workspace_size_validation():
    p = dm.make_params(32, 100, 1)
    # 64 dimensions: complex-plane matrices by default (5 passes x 4 KiB per instance), the real-equivalent
    # layout 1 on request (5 x 8 KiB)
    ws_cx = dm.workspace_size(8, 32, 32, 64, p)
    ws_re = dm.workspace_size(8, 32, 32, 64, dm.make_params(32, 100, 1, tile_config=2))
    assert ws_cx > 8 * 20 * 1024 and ws_re - ws_cx == 8 * 20 * 1024
    for args, msg in [((8, 32, 32, 8), "qam_order"), ((0, 32, 32, 64), "n_inst"), ((8, 0, 4, 16), "nt"),
                      ((8, 129, 129, 16), "nt > 128"), ((8, 4, 5000, 16), "nr")]:
        with pytest.raises(dm.DmalaError) as e:
            dm.workspace_size(*args, p)
        assert msg in str(e.value)
    with pytest.raises(dm.DmalaError):
        dm.workspace_size(8, 4, 4, 16, dm.make_params(0, 10, 1))
    with pytest.raises(dm.DmalaError):
        dm.workspace_size(8, 40, 40, 16, dm.make_params(16, 10, 1, precision="fp64"))
    # every automatic layout exists for 1..128 antennas
    for nt in (1, 3, 16, 17, 33, 48, 64, 65, 100, 128):
        assert dm.workspace_size(2, nt, nt, 16, p) > 0
    # explicit layouts: valid only for their dimension count
    assert dm.workspace_size(2, 64, 64, 64, dm.make_params(16, 10, 1, tile_config=4)) > 0
    with pytest.raises(dm.DmalaError):
        dm.workspace_size(2, 32, 32, 64, dm.make_params(16, 10, 1, tile_config=4))


def test_detect_rejects_bad_workspace_before_launch():
    L = dm.lib()
    p = dm.make_params(16, 10, 1)
    o = dm.Outputs()
    fake = ctypes.c_void_p(0x1000)
    need = dm.workspace_size(2, 4, 4, 16, p)
    st = L.dmala_detect(fake, fake, fake, 2, 4, 4, 16, None, ctypes.byref(p), ctypes.byref(o), None, need, None)
    assert st == -4 and "workspace" in dm.last_error()
    st = L.dmala_detect(fake, fake, fake, 2, 4, 4, 16, None, ctypes.byref(p), ctypes.byref(o), ctypes.c_void_p(0x10000), need - 1, None)
    assert st == -4 and "too small" in dm.last_error()
    st = L.dmala_detect(None, fake, fake, 2, 4, 4, 16, None, ctypes.byref(p), ctypes.byref(o), ctypes.c_void_p(0x10000), need, None)
    assert st == -1
    bad = (ctypes.c_float * 32)(*([0.5] * 32))
    st = L.dmala_detect(fake, fake, fake, 2, 4, 4, 16, bad, ctypes.byref(p), ctypes.byref(o), ctypes.c_void_p(0x10000), need, None)
    assert st == -2 and "constellation" in dm.last_error()


def _lparams(**kw):
    p = dm.make_params(16, 10, 1, proposal="learned")
    p.mlp_weights = 0x2000
    p.mix_eps = 0.1
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_learned_proposal_validation():
    assert dm.workspace_size(2, 8, 8, 16, _lparams()) > 0
    assert dm.workspace_size(2, 64, 64, 64, _lparams()) > 0            # 128 dims: layout 3
    for kw, msg in [(dict(mlp_weights=None), "mlp_weights"), (dict(mix_eps=1.5), "mix_eps"),
                    (dict(mix_eps=-0.1), "mix_eps"), (dict(precision=dm.FP64), "FP64")]:
        with pytest.raises(dm.DmalaError) as e:
            dm.workspace_size(2, 8, 8, 16, _lparams(**kw))
        assert msg in str(e.value)
    with pytest.raises(dm.DmalaError) as e:       # layout 2 (128 dims in one wave) is not built for it
        dm.workspace_size(2, 64, 64, 64, _lparams(tile_config=3))
    assert "tile_config" in str(e.value)


def test_train_rows_need_the_preconditioned_proposal():
    L = dm.lib()
    p = dm.make_params(16, 10, 1, proposal="naive")
    o = dm.Outputs()
    o.train_rows = 0x3000
    fake = ctypes.c_void_p(0x1000)
    need = dm.workspace_size(2, 4, 4, 16, p)
    st = L.dmala_detect(fake, fake, fake, 2, 4, 4, 16, None, ctypes.byref(p), ctypes.byref(o), ctypes.c_void_p(0x10000), need, None)
    assert st == -2 and "train_rows" in dm.last_error()


def test_mlp_entry_points_validate_on_the_host():
    L = dm.lib()
    f = ctypes.c_void_p(0x1000)
    assert L.dmala_mlp_forward(f, f, 10, 5, f, None) == -1 and "row_stride" in dm.last_error()
    assert L.dmala_mlp_forward(None, f, 10, 12, f, None) == -1
    assert L.dmala_mlp_train_workspace_size(0) == 0
    need = L.dmala_mlp_train_workspace_size(1000)
    assert need >= 1000 * 4 * 64
    ws = ctypes.c_void_p(0x10000)
    assert L.dmala_mlp_train_step(f, f, f, 1, 1e-3, f, f, 0, None, None, ws, need, None) == -1
    assert L.dmala_mlp_train_step(f, f, f, 0, 1e-3, f, f, 1000, None, None, ws, need, None) == -1
    assert L.dmala_mlp_train_step(f, f, f, 1, -1.0, f, f, 1000, None, None, ws, need, None) == -1
    assert L.dmala_mlp_train_step(f, f, f, 1, 1e-3, f, f, 1000, None, None, ws, need - 1, None) == -4
    assert L.dmala_mlp_train_step(f, f, f, 1, 1e-3, f, f, 1000, None, None, ctypes.c_void_p(0x10010), need, None) == -4


def test_learned_only_layouts():
    # layouts 5 and 6 (tile_config 6, 7) exist for the learned mixture only
    assert dm.workspace_size(2, 32, 32, 64, _lparams(tile_config=6)) > 0
    assert dm.workspace_size(2, 64, 64, 64, _lparams(tile_config=7)) > 0
    with pytest.raises(dm.DmalaError):
        dm.workspace_size(2, 32, 32, 64, dm.make_params(16, 10, 1, tile_config=6))
    with pytest.raises(dm.DmalaError):
        dm.workspace_size(2, 32, 32, 64, _lparams(tile_config=7))      # 64 dims, not 128
    with pytest.raises(dm.DmalaError):
        dm.workspace_size(2, 32, 32, 64, dm.make_params(16, 10, 1, tile_config=8))


def test_llr_mode_validation():
    p = dm.make_params(16, 10, 1, llr_mode="list")
    assert dm.workspace_size(2, 4, 4, 16, p) > 0
    p.llr_mode = 3
    with pytest.raises(dm.DmalaError) as e:
        dm.workspace_size(2, 4, 4, 16, p)
    assert "llr_mode" in str(e.value)


def test_detect_one_checks_sigma2_and_arguments_on_the_host():
    """dmala_detect_one refuses sigma^2 <= 0 or non-finite with DMALA_ERR_NONFINITE before any launch
    (Lemma 1 needs sigma^2 > 0), and validates the constellation and the workspace."""
    L = dm.lib()
    need = L.dmala_detect_one_workspace_size(4, 4, 16, 16)
    assert need >= dm.workspace_size(1, 4, 4, 16, dm.make_params(16, 10, 1)) + 256
    assert L.dmala_detect_one_workspace_size(4, 4, 8, 16) == 0
    f = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x10000)
    for s2 in (0.0, -1.0, float("nan"), float("inf")):
        st = L.dmala_detect_one(f, f, s2, 4, 4, None, 16, 16, 10, 1, f, None, ws, need, None)
        assert st == -3 and "sigma" in dm.last_error(), s2
    bad = (ctypes.c_float * 32)(*([0.5] * 32))
    assert L.dmala_detect_one(f, f, 0.1, 4, 4, bad, 16, 16, 10, 1, f, None, ws, need, None) == -2
    assert L.dmala_detect_one(f, f, 0.1, 4, 4, None, 16, 16, 10, 1, None, None, ws, need, None) == -1
    assert L.dmala_detect_one(f, f, 0.1, 4, 4, None, 16, 16, 10, 1, f, None, ws, need - 1, None) == -4
    assert L.dmala_detect_one(f, f, 0.1, 4, 4, None, 16, 16, 10, 1, f, None, ctypes.c_void_p(0x10010), need, None) == -4
    assert L.dmala_sync_status(None, 4, None) == -1
    assert L.dmala_sync_status(f, 0, None) == -1


def test_mhgd_proposal_validation():
    assert dm.workspace_size(2, 8, 8, 16, dm.make_params(16, 10, 1, proposal="mhgd")) > 0
    assert dm.workspace_size(2, 8, 8, 16, dm.make_params(16, 10, 1, proposal="mhgd", precision="bf16")) > 0
    assert dm.workspace_size(2, 8, 8, 16, dm.make_params(16, 10, 1, proposal="mhgd", precision="fp64")) > 0
    with pytest.raises(dm.DmalaError) as e:
        dm.workspace_size(2, 8, 8, 16, dm.make_params(16, 10, 1, proposal="mhgd", precision="fp16"))
    assert "MHGD" in str(e.value)
    L = dm.lib()
    p = dm.make_params(16, 10, 1, proposal="mhgd")
    o = dm.Outputs()
    o.train_rows = 0x3000
    fake = ctypes.c_void_p(0x1000)
    need = dm.workspace_size(2, 4, 4, 16, p)
    st = L.dmala_detect(fake, fake, fake, 2, 4, 4, 16, None, ctypes.byref(p), ctypes.byref(o), ctypes.c_void_p(0x10000),
                        need, None)
    assert st == -2 and "train_rows" in dm.last_error()
