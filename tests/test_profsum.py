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


@pytest.mark.parametrize("name", ["k_sweep_config4_257x16.txt", "k_sweep_levelpair65_33x64.txt"])
def test_committed_traffic_summary_is_readable(name):
    # the summaries bench.py reads its roofline traffic from: counter bytes
    # per launch, the copy calibration, and the hash of the sweep source they
    # were taken on (equal to the current source's, or bench.py reports no
    # traffic)
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                        name)
    rec = profsum.read_summary(path)
    assert rec["hbm_bytes_per_launch"] > 0
    assert len(rec["kernel_source_sha256"]) == 64
    assert rec["kernel_source_sha256"] == profsum.source_hash()
    assert rec["fetch_scale"] > 0 and rec["write_scale"] > 0
    json.dumps(rec)


def test_finest_sweeps_follow_the_v_cycle():
    # two batches of three cycles on two sweep levels (finest F, coarser C)
    # above a small-grid V-cycle; the finest grid's sweep kinds differ in
    # launch shape (the selection must not depend on it)
    def row(i, name):
        return {"Dispatch_Id": str(i), "Kernel_Name": name,
                "Start_Timestamp": str(10 * i), "End_Timestamp": str(10 * i + 5)}
    F = {"in": "k_sweep_res_in_cb<double, 8, 64, false>",
         "plain": "k_sweep<double, 8, 64, false, true, false>",
         "pro": "k_sweep<double, 16, 32, true, true, false>",
         "out": "k_sweep_res_out<double, 8, 64, true, false>"}
    C = {"in": "k_sweep_res_in<double, 16, 16, false>",
         "plain": "k_sweep<double, 16, 16, false, false, false>",
         "pro": "k_sweep<double, 8, 32, true, false, false>",
         "out": "k_sweep_res_out<double, 16, 16, false, false>"}
    seq, i = [], 0
    for _ in range(2):
        seq.append(row(i, "k_init_state(...)")); i += 1
        for _c in range(3):
            for nm in (F["in"], "k_finalize(...)", F["plain"], "k_resrestrict<double, 4, 32, true, false>",
                       C["in"], "k_finalize(...)", C["plain"], "k_resrestrict<double, 8, 16, false, false>",
                       "k_vsmall<double, 17>(...)", C["pro"], C["out"], F["pro"], F["out"]):
                seq.append(row(i, nm)); i += 1
        seq.append(row(i, "k_reduce(...)")); i += 1
    sel = profsum.finest_sweeps(seq, batches=1, cycles_upto=2)
    assert [(k, c) for k, c, _ in sel] == [(3, 1), (0, 1), (1, 1), (2, 1),
                                           (3, 2), (0, 2), (1, 2), (2, 2)]
    assert all(r["Kernel_Name"] in F.values() for _, _, r in sel)
    # the selected rows belong to the last batch
    assert min(int(r["Dispatch_Id"]) for _, _, r in sel) > 40
    assert len(profsum.finest_sweeps(seq, batches=2, cycles_upto=9)) == 2 * 3 * 4


def test_kernel_overlap_of_a_trace():
    def row(a, b):
        return {"Start_Timestamp": str(a), "End_Timestamp": str(b)}
    # [0,10) alone, [10,20) back to back (no overlap), [15,30) overlapping the
    # second by 5, [40,50) after a gap
    o = profsum.kernel_overlap([row(0, 10), row(10, 20), row(15, 30), row(40, 50)])
    assert o["kernels"] == 4
    assert o["busy_ns"] == 40 and o["span_ns"] == 50
    assert o["kernel_ns"] == 10 + 10 + 15 + 10
    assert abs(o["overlap_share"] - 5 / 40) < 1e-12
    assert abs(o["mean_concurrency"] - 45 / 40) < 1e-12
    assert profsum.kernel_overlap([])["busy_ns"] == 0
