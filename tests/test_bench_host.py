"""Host checks of bench.py's measurement helpers (no GPU).

The backward raster's work counter is run on a frame the oracle binned,
sorted and composited: every (pixel, record) visit it counts must be one of
the records before the pixel's last contributor, so the visits add up to the
sum of the contributor counts, and the counts are nested
(visits >= in-support >= contributing >= gradient terms)."""
import numpy as np
import pytest
import torch

import bench
from oracle import preprocess as opp
from oracle import raster as ora
from synth import make_config


class _Frame:
    """The workspace accessors the counter reads, over oracle arrays."""

    def __init__(self, rec32, vals, ranges, ncontrib):
        self._rec, self._vals, self._rg, self._nc = rec32, vals, ranges, ncontrib

    def records(self):
        return torch.tensor(self._rec)

    def ranges(self):
        return torch.tensor(self._rg.astype(np.int64))

    def sorted_pairs(self, n):
        return None, torch.tensor(self._vals[:n].astype(np.int64))

    def ncontrib(self):
        return torch.tensor(self._nc.reshape(-1).astype(np.int64))


@pytest.mark.parametrize("n,W,H", [(3000, 100, 70), (20000, 64, 48)])
def test_raster_work_counts_match_contributor_sums(n, W, H):
    cfg = make_config("headline", n=n, width=W, height=H)
    sc, v = cfg["scenes"][0], cfg["views"][0]
    rec = opp.preprocess(torch.tensor(sc.params.astype(np.float64)), sc.dim, sc.rot, v)["rec"]
    rec32 = rec.numpy().astype(np.float32)
    G = ((W + 15) // 16) * ((H + 15) // 16)
    keys, vals = ora.bin_view(rec32, W, H)
    _, sv, rg = ora.sort_and_ranges(keys, vals, G)
    _, _, nc, _ = ora.render_fwd(rec32.astype(np.float64), W, H)
    w = bench.raster_bwd_work(_Frame(rec32, sv, rg, nc), v, len(sv), chunk=257)
    assert w["eval"] == int(nc.sum()) == w["sum_ncontrib"]
    assert w["eval"] >= w["support"] >= w["contrib"] >= w["grad"] > 0
    assert w["pair"] == len(sv) >= w["pairs_active"] > 0
    assert w["lane_ops"] == sum(bench.BWD_OPS[k] * w[k] for k in bench.BWD_OPS)


def test_gpus_other_than_one_exit_with_message(capsys, monkeypatch):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    assert bench.main() == 2
    assert "one GPU" in capsys.readouterr().err


def test_cpu_baseline_reports_one_and_all_threads():
    cfg = make_config("cfg0", n=500, width=64, height=48)
    cb = bench.cpu_baseline(cfg, rows=8, sub=200, max_workers=2)
    assert cb["kind"] == "oracle" and cb["unit"] == "frames/s"
    assert cb["cores"] == min(2, cb["usable_cpus"])
    assert cb["value"] > 0 and cb["single_thread_value"] > 0
    assert cb["nproc"] >= 1 and isinstance(cb["cpu_model"], str)
