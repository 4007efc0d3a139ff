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
