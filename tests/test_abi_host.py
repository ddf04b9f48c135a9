"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/ubs.h, the ctypes structs match the C
structs byte for byte, the size query works and argument errors are reported
before any launch."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ubs.h")

lib_mod = pytest.importorskip("paper_2510_03312_amd._lib")
from paper_2510_03312_amd import _lib  # noqa: E402
from paper_2510_03312_amd.renderer import FrameDesc, SceneRef, Tuning  # noqa: E402
from synth import make_config, param_count  # noqa: E402


def _declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:ubs_status|int32_t)\s+(ubs_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_entry_point():
    L = _lib.load()
    names = _declared_functions()
    assert set(names) == set(_lib.EXPORTS)
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}$", out, re.M), n


def test_abi_version_and_param_counts():
    assert _lib.ubs_abi_version() == 2
    for dim in (3, 6, 7, 8, 9, 10):
        for rot in (0, 1):
            assert _lib.ubs_param_count(dim, rot) == param_count(dim, rot)
    assert _lib.ubs_param_count(10, 0) == 78
    assert _lib.ubs_param_count(11, 0) == 0
    assert _lib.ubs_param_count(6, 1) == 35
    assert _lib.ubs_param_count(7, 1) == 44
    assert _lib.ubs_param_count(5, 0) == 0


def test_ctypes_structs_match_the_header(tmp_path):
    prog = tmp_path / "sz.c"
    fields = {
        "ubs_scene": ["dim", "rot", "n", "params", "dparams"],
        "ubs_view": ["scene", "width", "height", "R", "t", "fx", "fy", "cx", "cy", "time", "query"],
        "ubs_tuning": ["tile_w", "tile_h", "batch_depth", "digit_bits", "pair_capacity", "flags",
                       "tile_slots"],
        "ubs_frame": ["scenes", "n_scenes", "n_views", "views", "tuning", "stage_events"],
        "ubs_layout": ["bytes", "n_records", "n_tiles", "n_pixels", "pair_capacity", "key_bits",
                       "n_views", "off_status", "off_records", "off_keys", "off_values",
                       "off_ranges", "off_ncontrib", "off_grad2d", "off_live"],
        "ubs_status_block": ["pairs_needed", "overflow", "n_nonfinite", "n_visible", "sort_stalled",
                             "spill"],
        "ubs_adam": ["lr_mu_x", "lr_opacity", "lr_scale", "lr_other", "beta1", "beta2", "eps",
                     "lambda_o", "lambda_s", "lambda_eps", "step"],
    }
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void){"]
    for s, fs in fields.items():
        lines.append(f'printf("{s} %zu\\n", sizeof({s}));')
        for f in fs:
            lines.append(f'printf("{s}.{f} %zu\\n", offsetof({s}, {f}));')
    lines.append("return 0;}")
    prog.write_text("\n".join(lines))
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(prog)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    py = {"ubs_scene": _lib.UbsScene, "ubs_view": _lib.UbsView, "ubs_tuning": _lib.UbsTuning,
          "ubs_frame": _lib.UbsFrame, "ubs_layout": _lib.UbsLayout,
          "ubs_status_block": _lib.UbsStatusBlock, "ubs_adam": _lib.UbsAdam}
    for s, fs in fields.items():
        assert int(got[s]) == ctypes.sizeof(py[s]), s
        for f in fs:
            assert int(got[f"{s}.{f}"]) == getattr(py[s], f).offset, (s, f)
    assert int(got["ubs_view"]) == 96
    src = open(HEADER).read()
    assert int(re.search(r"UBS_N_STAGES = (\d+)", src).group(1)) == _lib.N_STAGES


class _FakeTensor:
    """Just enough of a tensor for FrameDesc on a machine without a GPU."""

    def __init__(self, shape):
        self.shape = shape
        self.dtype = __import__("torch").float32

    def is_contiguous(self):
        return True

    def data_ptr(self):
        return 0x1000


def _frame(cfg, tuning=None, capacity=1 << 20):
    scenes = [SceneRef(_FakeTensor(s.params.shape), s.dim, s.rot) for s in cfg["scenes"]]
    return FrameDesc(scenes, cfg["views"], tuning or Tuning(), capacity)


def test_size_query_without_gpu():
    cfg = make_config("headline", n=1000, width=100, height=60)
    f = _frame(cfg)
    lay = _lib.UbsLayout()
    _lib.ubs_preprocess(f.c, 0, 0, lay, 0)
    assert lay.n_records == 1000
    assert lay.n_tiles == 7 * 4
    assert lay.n_pixels == 6000
    assert lay.key_bits == 32 + 5
    assert lay.pair_capacity == 1 << 20
    offs = [lay.off_status, lay.off_records, lay.off_keys, lay.off_values, lay.off_ranges,
            lay.off_ncontrib, lay.off_grad2d, lay.off_live]
    assert all(o % 256 == 0 for o in offs)
    assert lay.bytes >= lay.off_grad2d + 40 * 1000
    assert lay.bytes >= lay.off_live + 1000
    # multi-view frames concatenate records, tiles and pixels
    cfg4 = make_config("cfg4", scene_sizes=(10, 20, 30, 40), n_views=6)
    lay4 = _lib.UbsLayout()
    _lib.ubs_preprocess(_frame(cfg4).c, 0, 0, lay4, 0)
    assert lay4.n_records == sum(cfg4["scenes"][v.scene].n for v in cfg4["views"])
    assert lay4.n_pixels == sum(v.width * v.height for v in cfg4["views"])


@pytest.mark.parametrize("mutate,code", [
    (lambda f: setattr(f.c.tuning, "tile_w", 12), _lib.UBS_ERR_UNSUPPORTED),
    (lambda f: setattr(f.c.tuning, "digit_bits", 12), _lib.UBS_ERR_UNSUPPORTED),
    (lambda f: setattr(f.c.tuning, "batch_depth", 96), _lib.UBS_ERR_UNSUPPORTED),
    (lambda f: setattr(f.c.tuning, "pair_capacity", -1), _lib.UBS_ERR_ARG),
    (lambda f: setattr(f.c.tuning, "tile_slots", 128), _lib.UBS_ERR_UNSUPPORTED),
    (lambda f: setattr(f.c.tuning, "tile_slots", 300), _lib.UBS_ERR_UNSUPPORTED),
    (lambda f: setattr(f.c.tuning, "tile_slots", 4160), _lib.UBS_ERR_UNSUPPORTED),
    (lambda f: setattr(f._sc[0], "dim", 5), _lib.UBS_ERR_UNSUPPORTED),
    (lambda f: setattr(f._sc[0], "dim", 11), _lib.UBS_ERR_ARG),
    (lambda f: setattr(f._sc[0], "rot", 3), _lib.UBS_ERR_ARG),
    (lambda f: setattr(f._sc[0], "params", None), _lib.UBS_ERR_ARG),
    (lambda f: setattr(f._vw[0], "scene", 4), _lib.UBS_ERR_ARG),
    (lambda f: setattr(f._vw[0], "width", 0), _lib.UBS_ERR_ARG),
    (lambda f: setattr(f._vw[0], "fx", float("nan")), _lib.UBS_ERR_ARG),
    (lambda f: f._vw[0].query.__setitem__(2, float("inf")), _lib.UBS_ERR_ARG),
    (lambda f: setattr(f.c, "n_scenes", -1), _lib.UBS_ERR_ARG),
])
def test_argument_errors_are_reported_before_launch(mutate, code):
    cfg = make_config("cfg0", n=100, width=64, height=64)
    f = _frame(cfg)
    mutate(f)
    lay = _lib.UbsLayout()
    assert _lib.ubs_preprocess(f.c, 0, 0, lay, 0, check=False) == code
    # the other entry points validate the same frame the same way (a bogus,
    # never-dereferenced workspace pointer: validation fails first)
    assert _lib.ubs_bin_sort(f.c, 0x100, 1 << 30, 0, check=False) == code


def test_tile_slots_size_the_workspace():
    """Each tile's slot block takes tuning.tile_slots keys of 8 bytes (0: 256)."""
    cfg = make_config("cfg0", n=100, width=64, height=64)
    sizes = {}
    for slots in (0, 256, 1024, 4096):
        f = _frame(cfg)
        f.c.tuning.tile_slots = slots
        lay = _lib.UbsLayout()
        assert _lib.ubs_preprocess(f.c, 0, 0, lay, 0) == 0
        sizes[slots] = lay.bytes
    assert sizes[0] == sizes[256]
    assert sizes[1024] - sizes[256] == 16 * 768 * 8
    assert sizes[4096] - sizes[256] == 16 * 3840 * 8


def test_workspace_checks():
    cfg = make_config("cfg0", n=100, width=64, height=64)
    f = _frame(cfg)
    lay = _lib.UbsLayout()
    _lib.ubs_preprocess(f.c, 0, 0, lay, 0)
    # too small a workspace, misaligned workspace, null layout on a size query
    assert _lib.ubs_bin_sort(f.c, 0x1000, lay.bytes - 1, 0, check=False) == _lib.UBS_ERR_CAPACITY
    assert _lib.ubs_bin_sort(f.c, 0x1008, lay.bytes, 0, check=False) == _lib.UBS_ERR_ARG
    assert _lib.load().ubs_preprocess(ctypes.byref(f.c), None, 0, None, None) == _lib.UBS_ERR_ARG
    # render_bwd needs exactly one gradient input
    assert _lib.ubs_render_bwd(f.c, 0x1000, lay.bytes, 0, 0, 0, 0, 0, check=False) == _lib.UBS_ERR_ARG
    assert _lib.ubs_render_bwd(f.c, 0x1000, lay.bytes, 0x2000, 0, 0x3000, 0x4000, 0,
                               check=False) == _lib.UBS_ERR_ARG


def test_empty_frame_is_valid():
    f = _frame(make_config("cfg0", n=10, width=16, height=16))
    f.c.n_views = 0
    lay = _lib.UbsLayout()
    _lib.ubs_preprocess(f.c, 0, 0, lay, 0)
    assert lay.n_records == 0 and lay.n_pixels == 0 and lay.n_tiles == 0
    assert np.isfinite(lay.bytes)


@pytest.mark.parametrize("change,code", [
    (dict(step=0), _lib.UBS_ERR_ARG),
    (dict(beta1=1.0), _lib.UBS_ERR_ARG),
    (dict(beta2=-0.1), _lib.UBS_ERR_ARG),
    (dict(eps=-1.0), _lib.UBS_ERR_ARG),
    (dict(dim=5), _lib.UBS_ERR_UNSUPPORTED),
    (dict(dim=11), _lib.UBS_ERR_ARG),
    (dict(rot=2), _lib.UBS_ERR_ARG),
    (dict(n=-1), _lib.UBS_ERR_ARG),
    (dict(params=0), _lib.UBS_ERR_ARG),
    (dict(n=0, params=0), _lib.UBS_OK),   # nothing to do, nothing launched
])
def test_adam_step_argument_errors(change, code):
    from paper_2510_03312_amd.optim import AdamConfig
    a = dict(step=1, beta1=0.9, beta2=0.999, eps=1e-15, dim=7, rot=0, n=10, params=0x1000)
    a.update(change)
    cfg = AdamConfig(beta1=a["beta1"], beta2=a["beta2"], eps=a["eps"]).to_c(a["step"])
    got = _lib.ubs_adam_step(cfg, a["dim"], a["rot"], a["n"], a["params"], 0x2000, 0x3000,
                             0x4000, 0, 0, check=False)
    assert got == code


def test_relocate_size_query_and_errors():
    need = _lib.ubs_relocate(7, 0, 1000, 0, 0, 0, 0, 0.005, 0, 0, 0, 0, 0)
    assert need >= 1000 * (8 + 4 * 6)
    assert _lib.ubs_relocate(7, 0, 0, 0, 0, 0, 0, 0.005, 0, 0, 0, 0, 0) >= 0
    bad = [dict(dim=5, code=_lib.UBS_ERR_UNSUPPORTED), dict(rot=3, code=_lib.UBS_ERR_ARG),
           dict(n=-1, code=_lib.UBS_ERR_ARG), dict(o_min=-1.0, code=_lib.UBS_ERR_ARG),
           dict(ws_bytes=16, code=_lib.UBS_ERR_CAPACITY), dict(params=0, code=_lib.UBS_ERR_ARG)]
    for b in bad:
        a = dict(dim=7, rot=0, n=1000, params=0x1000, o_min=0.005, ws_bytes=need)
        a.update(b)
        got = _lib.ubs_relocate(a["dim"], a["rot"], a["n"], a["params"], 0x2000, 0x3000, 0x4000,
                                a["o_min"], 0x5000, a["ws_bytes"], 0, 0, 0, check=False)
        assert got == b["code"], b


def test_ssim_loss_size_query_and_errors():
    need = _lib.ubs_ssim_loss([(64, 48), (30, 20)], 0, 0, 0.2, 0, 0, 0, 0, 0)
    assert need >= (64 * 48 + 30 * 20) * 36
    cases = [(dict(sizes=[(0, 5)]), _lib.UBS_ERR_ARG), (dict(lam=1.5), _lib.UBS_ERR_ARG),
             (dict(ws_bytes=8), _lib.UBS_ERR_CAPACITY), (dict(image=0), _lib.UBS_ERR_ARG)]
    for change, code in cases:
        a = dict(sizes=[(64, 48)], lam=0.2, image=0x1000, ws_bytes=need)
        a.update(change)
        got = _lib.ubs_ssim_loss(a["sizes"], a["image"], 0x2000, a["lam"], 0x3000, 0, 0x4000,
                                 a["ws_bytes"], 0, check=False)
        assert got == code, change


def test_python_constants_match_the_header():
    src = open(HEADER).read()
    defs = dict(re.findall(r"^#define\s+(UBS_\w+)\s+(.+?)\s*(?:/\*.*)?$", src, re.M))
    for name in ("UBS_TUNE_PERSISTENT", "UBS_TUNE_PRE_FP32", "UBS_TUNE_NO_BETA_COND",
                 "UBS_TUNE_NO_BETA_OPACITY", "UBS_RELOCATE_NOALLOC_MAX_N"):
        assert eval(defs[name].replace("u", "")) == getattr(_lib, name), name


def test_noalloc_relocate_rejects_oversize_before_any_launch():
    big = _lib.UBS_RELOCATE_NOALLOC_MAX_N + 1
    assert _lib.ubs_relocate_noalloc(7, 0, big, 0, 0, 0, 0, 0.005, 0, 0, 0,
                                     check=False) == _lib.UBS_ERR_CAPACITY
    assert _lib.ubs_relocate_noalloc(5, 0, 10, 0, 0, 0, 0, 0.005, 0, 0, 0,
                                     check=False) == _lib.UBS_ERR_UNSUPPORTED
    assert _lib.ubs_relocate_noalloc(7, 0, 10, 0, 0, 0, 0, 0.005, 0, 0, 0,
                                     check=False) == _lib.UBS_ERR_ARG
    assert _lib.ubs_relocate_noalloc(7, 0, 0, 0, 0, 0, 0, 0.005, 0, 0, 0,
                                     check=False) == _lib.UBS_OK
