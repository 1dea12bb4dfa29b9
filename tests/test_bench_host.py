"""Host logic of bench.py's rocprofv3 summaries: kernel names map to kernel families
without double counting, for every type configuration the library instantiates."""
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

CFGS = ["lv::Cfg<int, int, long, int>", "lv::Cfg<int, long, __int128, long>",
        "lv::Cfg<int, long, __int128, int>", "lv::Cfg<long, long, __int128, long>"]


def families_of(name):
    return [f for f, pats in bench.FAMILY_KERNELS.items() if any(re.search(p, name) for p in pats)]


def test_profiled_kernels_map_to_at_most_one_family():
    data = json.load(open(os.path.join(ROOT, "profiles", "rmat24_fast_pmc.json")))
    for name in data["kernels"]:
        assert len(families_of(name)) <= 1, name
    fams = data["families"]
    assert "move_bin6_hub" in fams and "agg_bin6_hub" in fams
    for f, rec in fams.items():
        assert rec["launches"] > 0 and rec["bytes_per_launch"] > 0, f


def test_every_configuration_maps_to_its_family():
    ns = "void lv::(anonymous namespace)::"
    for cfg in CFGS:
        wide = "__int128" in cfg
        cases = {
            "k_move_wave<%s, 1, 8, 4, true>" % cfg: "move_bin0_1lane",
            "k_move_wave<%s, 16, 8, 8, false>" % cfg: "move_bin2_16lanes",
            "k_move_wave<%s, 64, 8, 10, true>" % cfg: "move_bin3_wave",
            "k_move_block<%s, 512, true>" % cfg: "move_bin5_bigblock",
            "k_hub_part<%s >" % cfg: "move_bin6_hub",
            "k_agg_wave<%s, 4, 4>" % cfg: "agg_bin0_4lanes",
            "k_agg_wave<%s, 4, 6>" % cfg: "agg_bin1_4lanes",
            "k_agg_wave<%s, %d, 8>" % (cfg, 16 if wide else 8): "agg_bin2_8lanes",
            "k_agg_hub_count<%s, int>" % cfg: "agg_bin6_hub",
        }
        for kernel, fam in cases.items():
            assert families_of(ns + kernel + "(args)") == [fam], kernel


def test_copy_probe_calibration_is_recorded():
    data = json.load(open(os.path.join(ROOT, "profiles", "rmat24_fast_pmc.json")))
    # FETCH_SIZE counts half of what a plain copy reads on this part; WRITE_SIZE all it writes
    assert abs(data["fetch_factor"] - 2.0) < 0.05 and abs(data["write_factor"] - 1.0) < 0.05


def test_pmc_summary_is_of_the_current_sources():
    # the default line reads its traffic from this summary only while the sources it was
    # measured on are the ones in the tree (else it reports traffic null)
    data = json.load(open(os.path.join(ROOT, "profiles", "rmat24_fast_pmc.json")))
    assert data["workload"] == "rmat24"
    assert data["sources_sha256"] == bench.sources_digest()
    fam = bench.measured_traffic("move_bin6_hub", os.path.join(ROOT, "profiles", "rmat24_fast_pmc.json"),
                                 workload="rmat24")
    assert fam is not None and fam > 0


def test_default_arguments(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert (a.gpus, a.steps, a.warmup, a.workload, a.mode) == (1, 5, 2, "rmat24", "fast")
    assert a.round_bits is None and a.q_runs == 0 and a.small_level == 0 and a.batch == 0
