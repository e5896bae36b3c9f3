"""Host logic of the counter summaries (paper_1004_1122_amd/profiling.py) on
synthetic rocprofv3 records: the marker windows that cut a run to one form's
timed launches, the per-dispatch means and the VALU issue-time model."""

import csv
import json
import re
import sys

from paper_1004_1122_amd import profiling


def _write_counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_issue_summary_windows_and_model(tmp_path, monkeypatch):
    d = tmp_path / "sq"
    d.mkdir()
    rows = []

    def disp(i, name, **vals):
        for c, v in vals.items():
            rows.append({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": c, "Counter_Value": v})

    marker = "void at::native::AbsFunctor<float>"
    row64, row32 = "void lshom::w3_row_kernel<double, 243, 0>(x)", "void lshom::w3_row_kernel<float, 243, 0>(x)"
    disp(1, row64, SQ_WAVES=1, SQ_INSTS_VALU=1)          # before the first window: ignored
    disp(2, marker, SQ_WAVES=1, SQ_INSTS_VALU=1)
    disp(3, row64, SQ_WAVES=100, SQ_INSTS_VALU=1000 * 100)
    disp(4, row64, SQ_WAVES=100, SQ_INSTS_VALU=1200 * 100)
    disp(5, marker, SQ_WAVES=1, SQ_INSTS_VALU=1)
    disp(6, marker, SQ_WAVES=1, SQ_INSTS_VALU=1)
    disp(7, row32, SQ_WAVES=50, SQ_INSTS_VALU=800 * 50)
    disp(8, marker, SQ_WAVES=1, SQ_INSTS_VALU=1)
    _write_counters(d / "run_counter_collection.csv", rows)
    passes = tmp_path / "pass.json"
    passes.write_text(json.dumps({"forms": {"fp64": {"passes": {"row": {"ms": 0.2}}},
                                            "mixed": {"passes": {"row": {"ms": 0.1}}}}}))
    out = tmp_path / "issue.md"
    monkeypatch.setattr(sys, "argv", [
        "profiling", "issue", "--dir", str(d), "--passes", str(passes), "--kernel",
        r"row=w3_row_kernel<{t}, 243, 0>", "--counters", "SQ_WAVES,SQ_INSTS_VALU", "--simds", "4",
        "--clock-ghz", "1.0", "--title", "t", "--command", "c", "--out", str(out)])
    profiling.main()
    text = out.read_text()
    rec = json.loads(re.search(r"^issue-json: (.*)$", text, re.M).group(1))
    fp64, mixed = rec["passes"]
    assert fp64["form"] == "fp64" and fp64["dispatches"] == 2 and fp64["SQ_WAVES"] == 100
    assert fp64["SQ_INSTS_VALU"] == 110000
    assert mixed["form"] == "mixed" and mixed["dispatches"] == 1 and mixed["SQ_INSTS_VALU"] == 40000
    # 110000 instructions x 4 cycles / (4 SIMDs x 1 GHz) = 110 us against a 200 us pass
    assert "| fp64 | row | 200.0 | 100 | 1100 | 0 | 110.0 | 0.55 |" in text
    assert "| mixed | row | 100.0 | 50 | 800 | 0 | 40.0 | 0.40 |" in text


def test_code_only_hash_ignores_comments():
    a = "int f(int x) {  // one\n  return x + 1; /* two */\n}\n"
    b = "// header\nint f(int x) {\n\n  return x + 1;\n}\n"
    c = "int f(int x) {\n  return x + 2;\n}\n"
    s = 'const char* p = "a // b";\n'
    assert profiling.code_only(a) == profiling.code_only(b)
    assert profiling.code_only(a) != profiling.code_only(c)
    assert profiling.code_only(s) == s.strip()
