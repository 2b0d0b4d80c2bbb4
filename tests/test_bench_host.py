"""Host-side checks of the benchmark script (no GPU): the one-GPU contract and the rule that reports the
committed HBM traffic only for the kernel sources and tilings (segment length, store policy of the stage
outputs, tile order) it was measured on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stdout


def test_traffic_only_for_the_measured_sources_and_tiling(monkeypatch):
    if not os.path.exists(bench.TRAFFIC_FILE):  # counters not taken: no traffic figure
        assert bench.measured_traffic("fp64", 64) is None and bench.measured_traffic("fp32c", 64) is None
        return
    text = open(bench.TRAFFIC_FILE).read()
    fields = dict(line.split(":", 1) for line in text.splitlines() if line.startswith("traffic_"))
    entries = []  # (tag, segment rows, store policy, tile order), figure
    for k, v in fields.items():
        if k.startswith("traffic_bytes_per_launch_"):
            tag, rest = k[len("traffic_bytes_per_launch_"):].split("_seg")
            seg, pol, ordr = rest.replace("_pol", " ").replace("_ord", " ").split()
            entries.append(((tag, int(seg), int(pol), int(ordr)), v))
    assert entries
    current = fields["traffic_source_hash"].strip() == bench.kernel_source_hash()
    seg_axis = int(fields["traffic_seg_axis_fp32c"])
    keys = {e[0] for e in entries}
    for (tag, seg, pol, ordr), v in entries:
        sa = seg_axis if tag == "fp32c" else 0
        t = bench.measured_traffic(tag, seg, sa, pol, ordr)
        if tag == "fp32c":  # another near-axis segment length: no figure
            assert bench.measured_traffic(tag, seg, seg_axis + 1, pol, ordr) is None
        for other in ((tag, seg, 1 - pol, ordr), (tag, seg, pol, 1 - ordr)):  # a tiling not measured: none
            if other not in keys:
                assert bench.measured_traffic(tag, seg, sa, other[2], other[3]) is None
        if current:  # counters taken on these sources
            assert t == int(float(v)) and t > 0
        else:  # the kernel changed since: no traffic figure until the counters are taken again
            assert t is None
    # a tiling without counters, or other sources: no traffic figure
    (tag, seg, pol, ordr), _ = entries[0]
    assert bench.measured_traffic(tag, 3 * seg, 0, pol, ordr) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic(tag, seg, seg_axis if tag == "fp32c" else 0, pol, ordr) is None
