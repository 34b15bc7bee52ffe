"""Host logic of the measurement tools: the request-counter summary and the
bench's reading of it (synthetic counter files, no GPU)."""
import csv
import importlib
import io
import os
import sys
from contextlib import redirect_stdout

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2204_10822_amd import profsum  # noqa: E402

FIELDS = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]


def _csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_requests_bytes(tmp_path):
    """Each request counts at its own size: 128/64/32-B reads, 64-B writes and the
    rest of the write requests at 32 B; means over dispatches."""
    k = "void vp::k_cheb_walk4<0, float>(int, float const*)"
    rd = tmp_path / "rd.csv"
    wr = tmp_path / "wr.csv"
    _csv(rd, [(k, 64, "TCC_EA0_RDREQ_sum", 1300000), (k, 64, "TCC_EA0_RDREQ_128B_sum", 1000000),
              (k, 64, "TCC_EA0_RDREQ_64B_sum", 200000), (k, 64, "TCC_EA0_RDREQ_32B_sum", 100000),
              (k, 64, "TCC_EA0_RDREQ_sum", 2600000), (k, 64, "TCC_EA0_RDREQ_128B_sum", 2000000),
              (k, 64, "TCC_EA0_RDREQ_64B_sum", 400000), (k, 64, "TCC_EA0_RDREQ_32B_sum", 200000)])
    _csv(wr, [(k, 64, "TCC_EA0_WRREQ_sum", 700000), (k, 64, "TCC_EA0_WRREQ_64B_sum", 400000)])
    out = io.StringIO()
    with redirect_stdout(out):
        profsum.requests(str(rd), str(wr))
    line = [l for l in out.getvalue().splitlines() if l.startswith("k_cheb_walk4<0, float>")][0]
    parts = line.rsplit(None, 10)
    n, r128, r64, r32, rmb, w64, w32, wmb, tot = parts[1:10]
    assert int(n) == 2
    assert (float(r128), float(r64), float(r32)) == (1500000.0, 300000.0, 150000.0)
    assert abs(float(rmb) - 216.0) < 0.006            # (128 * 1.5e6 + 64 * 3e5 + 32 * 1.5e5) / 1e6
    assert (float(w64), float(w32)) == (400000.0, 300000.0)
    assert abs(float(wmb) - 35.2) < 0.006             # (64 * 4e5 + 32 * 3e5) / 1e6
    assert abs(float(tot) - 251.2) < 0.006


def test_bench_reads_request_summary(tmp_path, monkeypatch):
    """bench.py takes `traffic` from the request summary's total column."""
    bench = importlib.import_module("bench")
    prof = tmp_path / "profiles"
    prof.mkdir()
    hdr = f"{'kernel':58s} {'n':>5s}\n"
    (prof / "vp_sharp_2048_kernels_requests.txt").write_text(
        "# synthetic\n" + hdr +
        f"{'k_cheb_walk4<0, float>':58s} {20:5d} {4554636:11.0f} {4486:9.0f} {0:9.0f} {583.28:9.2f} "
        f"{1030656:10.0f} {151554:9.0f} {70.81:9.2f} {654.09:9.2f} {127872:>10d}\n")
    monkeypatch.setattr(bench, "PROFILES", str(prof))
    traffic, raw = bench.counter_traffic("k_cheb_walk4<0, float>")
    assert abs(traffic - 654.09e6) < 1.0
    assert raw is None
    assert bench.counter_traffic("k_missing") == (None, None)
