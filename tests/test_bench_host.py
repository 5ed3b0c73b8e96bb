"""Host-side logic of bench.py (CPU only): the HBM traffic summary from
counter CSVs, and the source hash that decides whether stored counter values
still describe the kernels."""
import csv
import json
import os
import shutil

import bench

HEAD = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
NAMES = {
    "reference": "neg_kernel_vectorized4_kernel",
    "pass1": "void (anonymous namespace)::pass_kernel<float, 4096, 16, 1, 16, true, false, false, 0>(PassArgs)",
    "pass2": "void (anonymous namespace)::pass_kernel<float, 4096, 16, 2, 16, true, false, false, 0>(PassArgs)",
    "axis": "void (anonymous namespace)::pass_kernel<float, 256, 16, 3, 16, false, false, false, 0>(PassArgs)",
}


def write_csv(path, counter, kib):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEAD)
        i = 0
        for role, vals in kib.items():
            for v in vals:
                w.writerow([i, NAMES[role], counter, v])
                i += 1
            w.writerow([i, "some_other_kernel", counter, 1.0])  # ignored
            i += 1


def test_traffic_summary_scales_by_reference(tmp_path):
    log2n = 10
    n = 1 << log2n
    known = 8.0 * n  # bytes each way of the reference kernel
    # the fetch counter reads half the bytes (factor 2), the write counter all of them
    fetch = {"reference": [known / 2 / 1024] * 2, "pass1": [1.5 * known / 2 / 1024] * 3,
             "pass2": [known / 2 / 1024], "axis": [known / 2 / 1024] * 4}
    write = {"reference": [known / 1024] * 2, "pass1": [known / 1024] * 3,
             "pass2": [1.25 * known / 1024], "axis": [known / 1024] * 4}
    fc, wc, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "traffic.txt"
    write_csv(fc, "FETCH_SIZE", fetch)
    write_csv(wc, "WRITE_SIZE", write)
    rec = bench.summarize_counters(str(fc), str(wc), log2n, str(out))
    assert abs(rec["reference"]["fetch_scale"] - 2.0) < 1e-12
    assert abs(rec["reference"]["write_scale"] - 1.0) < 1e-12
    k = rec["kernels"]
    assert abs(k["pass1"]["fetch_bytes"] - 1.5 * known) < 1e-6
    assert abs(k["pass1"]["ratio_to_algorithmic"] - 1.25) < 1e-12
    assert abs(k["pass2"]["ratio_to_algorithmic"] - 1.125) < 1e-12
    assert abs(k["axis"]["ratio_to_algorithmic"] - 1.0) < 1e-12
    assert k["pass1"]["dispatches"] == [3, 3] and k["axis"]["dispatches"] == [4, 4]
    assert json.load(open(out))["source_hash"] == bench.kernel_source_hash()


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    src = os.path.join(bench.ROOT, "paper_0811_2535_amd", "csrc")
    fake = tmp_path / "paper_0811_2535_amd" / "csrc"
    fake.mkdir(parents=True)
    for f in ("liftfft.hip", "fft_engine.hpp"):
        shutil.copy(os.path.join(src, f), fake / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    p = fake / "liftfft.hip"
    text = p.read_text()
    p.write_text("// a new comment line\n/* and a block\n comment */\n" + text.replace("\n", "\n\n", 3) + "\n")
    assert bench.kernel_source_hash() == h0
    p.write_text(text.replace("constexpr int AXIS_WIDE_LMIN = 9;", "constexpr int AXIS_WIDE_LMIN = 10;"))
    assert bench.kernel_source_hash() != h0


def test_kernel_roles():
    assert bench._kernel_role(NAMES["pass1"]) == "pass1"
    assert bench._kernel_role(NAMES["pass2"]) == "pass2"
    assert bench._kernel_role(NAMES["axis"]) == "axis"
    assert bench._kernel_role(NAMES["reference"]) == "reference"
    assert bench._kernel_role("void pass_kernel<double, 256, 16, 3, 16>") is None
