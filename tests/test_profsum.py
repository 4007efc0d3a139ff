"""Host logic of the profile summaries: the kernel-source hash that ties the
HBM-traffic counters to the code they were taken on, and the JSON block that
bench.py reads back."""
import json
import os

import pytest

from paper_1607_03252_amd import profsum


def _src(tmp_path, body):
    p = tmp_path / "k.hip"
    p.write_text(body + "\n" + profsum.SWEEP_END.decode() + "\nint tail_changes_do_not_count;\n")
    return str(p)


def test_hash_ignores_comments_and_blank_space(tmp_path):
    a = _src(tmp_path, "// a comment\nint f(int x) {  return x + 1; }  /* block */\n")
    ha = profsum.source_hash(a)
    b = _src(tmp_path, "// another comment\n\nint f(int x) {\n  return x + 1;\n}\n")
    assert profsum.source_hash(b) == ha


def test_hash_follows_code_changes(tmp_path):
    a = _src(tmp_path, "int f(int x) { return x + 1; }\n")
    ha = profsum.source_hash(a)
    b = _src(tmp_path, "int f(int x) { return x + 2; }\n")
    assert profsum.source_hash(b) != ha


def test_hash_covers_only_the_sweep_section(tmp_path):
    p = tmp_path / "k.hip"
    head = "int f(int x) { return x; }\n" + profsum.SWEEP_END.decode() + "\n"
    p.write_text(head + "int g;\n")
    h1 = profsum.source_hash(str(p))
    p.write_text(head + "int h;\n")
    assert profsum.source_hash(str(p)) == h1


def test_committed_traffic_summary_is_readable():
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                        "k_sweep_traffic_levelpair65_33x64.txt")
    if not os.path.exists(path):
        pytest.skip("no traffic summary committed")
    rec = profsum.read_summary(path)
    assert rec["hbm_bytes_per_launch"] > 0
    assert len(rec["kernel_source_sha256"]) == 64
    assert rec["fetch_scale"] > 0 and rec["write_scale"] > 0
    json.dumps(rec)


def test_finest_sweeps_groups_the_largest_launches_by_cycle():
    # two batches; each cycle: two sweeps on the finest grid, a transfer, a
    # coarser grid's sweeps, two more finest sweeps (the first is judged)
    def row(i, name, grid):
        return {"Dispatch_Id": str(i), "Kernel_Name": name, "Grid_Size_X": str(grid),
                "Start_Timestamp": str(10 * i), "End_Timestamp": str(10 * i + 5)}
    seq, i = [], 0
    for _ in range(2):
        seq.append(row(i, "k_init_state(...)", 256)); i += 1
        for _c in range(3):
            for nm, g in (("k_sweep_res_in_cb<double, 16, 32, false>", 900),
                          ("k_finalize(...)", 4096),
                          ("k_sweep<double, 16, 32, false, true, false>", 900),
                          ("k_resrestrict<double, 4, 32, true, false>", 9000),
                          ("k_sweep<double, 16, 32, false, false, false>", 100),
                          ("k_sweep<double, 16, 32, true, true, false>", 900),
                          ("k_sweep_res_out<double, 16, 32, true, false>", 900)):
                seq.append(row(i, nm, g)); i += 1
    sel = profsum.finest_sweeps(seq, batches=1, cycles_upto=2)
    assert [(k, c) for k, c, _ in sel] == [(3, 1), (0, 1), (1, 1), (2, 1),
                                           (3, 2), (0, 2), (1, 2), (2, 2)]
    # the selected rows belong to the last batch
    assert min(int(r["Dispatch_Id"]) for _, _, r in sel) > 22
