"""The push counter summaries under profiles/ are written by
bench.py --summarize-push-pmc from rocprofv3 CSV output: on synthetic counter
files of known values it must derive the busy fractions, per-step rates and
calibrated HBM bytes by hand-checkable formulas, and the committed summary must
belong to the current push sources."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

PUSH = "void gc::k_push<0, 1, 0, true>(gc::PushArgs)"
COPY = "gc::k_copy_probe(uint4*, uint4 const*, unsigned long)"
FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]

# two push launches; every counter of launch L (1, 2) is L times its base value
BASE = {"SQ_INSTS_VALU": 1.8e9, "SQ_ACTIVE_INST_VALU": 1.0e9, "GRBM_GUI_ACTIVE": 8.0e7, "TA_TA_BUSY_sum": 6.4e8,
        "TD_TD_BUSY_sum": 7.2e8, "TA_FLAT_READ_WAVEFRONTS_sum": 1.0e8, "TCP_TOTAL_CACHE_ACCESSES_sum": 2.3e9,
        "TCP_TCC_READ_REQ_sum": 2.0e6, "SQ_INSTS_VALU_FLOPS_FP64": 1.5e9, "SQ_INSTS_VALU_CVT": 3.0e8,
        "SQ_INSTS_VALU_FMA_F64": 6.0e8, "SQ_INSTS_VALU_MUL_F64": 2.5e8, "SQ_INSTS_VALU_ADD_F64": 1.0e8,
        "SQ_INSTS_VALU_TRANS_F64": 2.0e7, "SQ_INSTS_VALU_INT32": 7.0e7, "SQ_INSTS_VALU_INT64": 2.0e7,
        "FETCH_SIZE": 6.0e4, "WRITE_SIZE": 1.2e5, "TCC_HIT_sum": 1.8e6, "TCC_MISS_sum": 1.2e6}
STEPS_PER_LAUNCH = 1.0e8


def _write_pass(d, name, counters):
    os.makedirs(os.path.join(d, f"pmc_{name}"))
    rows = []
    for disp, launch in ((1, None), (2, 1), (3, 2)):
        for c in counters:
            if launch is None:         # the copy probe first: 256 MiB read, 256 MiB written
                kn, v = COPY, {"FETCH_SIZE": 131072.0, "WRITE_SIZE": 262144.0}.get(c, 1.0)
            else:
                kn, v = PUSH, BASE[c] * launch
            # counters of some blocks come as several rows (per XCD): split them in two
            for part in (0.25, 0.75):
                rows.append({"Dispatch_Id": disp, "Kernel_Name": kn, "Counter_Name": c, "Counter_Value": v * part})
    with open(os.path.join(d, f"pmc_{name}", "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS, restval="0")
        w.writeheader()
        w.writerows(rows)
    line = {"metric": "m", "value": 1.0, "config": {"field_store": "f32", "precision": "f64"},
            "roofline": {"launches": 2, "particle_steps_per_launch": STEPS_PER_LAUNCH}}
    with open(os.path.join(d, f"pmc_{name}.log"), "w") as f:
        f.write("[bench] noise\n" + json.dumps(line) + "\n")


def test_summary_formulas(tmp_path):
    src = tmp_path / "runs"
    out = tmp_path / "out"
    out.mkdir()
    for name, counters in bench.PMC_PASSES.items():
        _write_pass(str(src), name, [c for c in counters.split() if c in BASE])
    valu, traffic = bench.summarize_push_pmc(str(src), out_dir=str(out))
    steps = 2 * STEPS_PER_LAUNCH
    s3 = 3.0                                   # launches 1 + 2
    cycles = s3 * BASE["GRBM_GUI_ACTIVE"] / 8  # GRBM summed over 8 XCDs
    assert valu["particle_steps"] == steps and valu["launches"] == 2
    assert valu["valu_instructions_per_particle_step"] == pytest.approx(s3 * 1.8e9 / steps)
    assert valu["valu_busy"] == pytest.approx(s3 * 1.0e9 / (256 * cycles))
    assert valu["ta_busy"] == pytest.approx(s3 * 6.4e8 / (256 * cycles))
    assert valu["td_busy"] == pytest.approx(s3 * 7.2e8 / (256 * cycles))
    assert valu["fp64_flops_per_particle_step"] == pytest.approx(64 * s3 * 1.5e9 / steps)
    assert valu["l1_tag_accesses_per_load"] == pytest.approx(23.0)
    # FETCH_SIZE scaled by 262144 / 131072 = 2, WRITE_SIZE by 1, KiB -> bytes
    assert traffic["fetch_scale"] == pytest.approx(2.0) and traffic["write_scale"] == pytest.approx(1.0)
    assert traffic["hbm_bytes_per_particle_step"] == pytest.approx(1024 * s3 * (2 * 6.0e4 + 1.2e5) / steps)
    assert traffic["l2_hit_rate"] == pytest.approx(0.6)
    assert valu["kernel_hash"] == bench.kernel_hash() == traffic["kernel_hash"]
    for fn in ("push_valu.json", "push_traffic.json", "push_f64_f32field_paper_scale_valu.md",
               "push_f64_f32field_paper_scale_traffic.md"):
        assert (out / fn).exists()


def test_launch_count_mismatch_is_refused(tmp_path):
    src = tmp_path / "runs"
    for name, counters in bench.PMC_PASSES.items():
        _write_pass(str(src), name, [c for c in counters.split() if c in BASE])
    line = {"metric": "m", "config": {"field_store": "f32", "precision": "f64"},
            "roofline": {"launches": 3, "particle_steps_per_launch": STEPS_PER_LAUNCH}}
    (src / "pmc_p1.log").write_text(json.dumps(line) + "\n")
    with pytest.raises(ValueError):
        bench.summarize_push_pmc(str(src), out_dir=str(tmp_path))


def test_committed_summary_belongs_to_the_push_sources():
    with open(os.path.join(ROOT, "profiles", "push_valu.json")) as f:
        valu = json.load(f)
    with open(os.path.join(ROOT, "profiles", "push_traffic.json")) as f:
        traffic = json.load(f)
    assert valu["kernel_hash"] == traffic["kernel_hash"] == bench.kernel_hash()
    assert 0.0 < valu["valu_busy"] <= 1.0 and 0.0 < valu["ta_busy"] <= 1.0


def test_launch_groups_cover_every_launch_once():
    assert bench._launch_groups(8) == [(i, i + 1) for i in range(8)]
    for n in (13, 100, 331, 1000):
        g = bench._launch_groups(n)
        assert len(g) == 10 and g[0][0] == 0 and g[-1][1] == n
        assert all(a < b for a, b in g) and all(g[i][1] == g[i + 1][0] for i in range(9))


def test_group_sums_and_busy_fractions():
    launches = [{"SQ_INSTS_VALU": 10.0 * (i + 1), "SQ_ACTIVE_INST_VALU": 5.0 * (i + 1), "GRBM_GUI_ACTIVE": 8.0,
                 "TA_TA_BUSY_sum": 2.0, "TD_TD_BUSY_sum": 3.0} for i in range(4)]
    g = bench._group_sums(launches, 1, 3)
    assert g["label"] == "2–3" and g["SQ_INSTS_VALU"] == 50.0 and g["GRBM_GUI_ACTIVE"] == 16.0
    cu_cycles = 256 * 16.0 / 8
    assert g["valu_busy"] == pytest.approx(25.0 / cu_cycles)
    assert g["ta_busy"] == pytest.approx(4.0 / cu_cycles) and g["td_busy"] == pytest.approx(6.0 / cu_cycles)
    assert bench._group_sums(launches, 2, 3)["label"] == "3"
